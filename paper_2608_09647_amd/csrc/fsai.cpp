// fsai.cpp -- preconditioned CG with M^-1 = G^T G, and the learned factor.
//
// The solve is the CG recurrence of Algorithm 1 with the preconditioned
// residual z = G^T (G r): rho = r^T z drives alpha and beta, the stop test
// stays on ||r|| / ||b||.  One iteration is four kernels on the stream:
//   q = A p (p^T q partials); x += alpha p, r -= alpha q with t = G r in the
//   same kernel (r^T r partials; G rows of at most 8 entries, else two
//   kernels); z = G^T t (r^T z partials); p = z + beta p (stop test).
// As in the unpreconditioned solve every scalar is reduced from the previous
// kernel's per-workgroup partials, so alpha, beta and the decisions never
// leave the device; the host polls the state every check_every iterations.
//
// The learned factor's values come from the network on the device
// (kernels_fsai.hip); the host only builds the structure (tril(A), its
// transpose, and the slot-to-position maps) once per handle.
#include <omp.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <utility>
#include <new>
#include <vector>

#include "../../include/cgmi_fsai.h"
#include "cgmi_host.h"
#include "fsai_internal.h"

using namespace cgmi;

#define HIP_TRY(expr) CGMI_HIP_TRY(expr)

// Learned-factor workspace of a handle; the structure is reused by later
// cg_fsai_setup calls with other parameters.
struct FsaiSetup {
    int32_t *d_scol = nullptr;   // n x 5 slot columns
    float *d_sval = nullptr;     // n x 5 A_hat values
    double *d_diag = nullptr;    // n
    uint16_t *d_feats = nullptr; // n x 16 bfloat16
    int32_t *d_err = nullptr;
    float *d_theta = nullptr;    // kNParams
    int32_t *d_gpos = nullptr;   // n x 3
    int32_t *d_tpos = nullptr;   // nnz(G)
};

namespace {

// Host array left uninitialised on allocation (its pages are first touched by
// the parallel loops that fill it, not by one thread zeroing it).
template <class T>
struct HostArray {
    std::unique_ptr<T[]> p;
    size_t n = 0;
    void alloc(size_t k) {
        p.reset(k ? new T[k] : nullptr);
        n = k;
    }
    T *data() { return p.get(); }
    const T *data() const { return p.get(); }
    size_t size() const { return n; }
    T &operator[](size_t i) { return p[i]; }
    const T &operator[](size_t i) const { return p[i]; }
};

struct HostCsr {
    HostVec<int32_t> rp;
    HostArray<int32_t> ci;
    HostArray<double> val;
};

// Transpose of an n x n CSR (columns of the result ascending); pos[k] is the
// position of input entry k in the result.  Host threads count the entries
// of every column and scatter them (atomic cursors), then sort each result
// row by column, so the layout does not depend on thread timing.  T.val is
// left empty when val is null.
void transpose(int32_t n, const int32_t *rp, const int32_t *ci, const double *val, HostCsr &T,
               HostArray<int32_t> *pos) {
    const int64_t nnz = rp[n];
    T.rp.resize((size_t)n + 1);
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j <= n; ++j) T.rp[j] = 0;
    T.ci.alloc((size_t)nnz);
    T.val.alloc(val ? (size_t)nnz : 0);
    if (pos) pos->alloc((size_t)nnz);
    HostArray<int32_t> src, next;
    src.alloc((size_t)nnz);
    next.alloc((size_t)n);
    int32_t *cnt = T.rp.data();
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nnz; ++k) __atomic_fetch_add(&cnt[ci[k] + 1], 1, __ATOMIC_RELAXED);
    par_running_sum(T.rp.data(), n);
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < n; ++j) next[j] = T.rp[j];
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t p = __atomic_fetch_add(&next[ci[k]], 1, __ATOMIC_RELAXED);
            T.ci[p] = i;
            src[p] = k;
        }
    // rows of the result by ascending column: insertion sort for short rows,
    // a comparison sort for long ones (a dense column of the input)
#pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t j = 0; j < n; ++j) {
        const int32_t r0 = T.rp[j], r1 = T.rp[j + 1];
        if (r1 - r0 > 32) {
            std::vector<std::pair<int32_t, int32_t>> e((size_t)(r1 - r0));
            for (int32_t a = r0; a < r1; ++a) e[(size_t)(a - r0)] = {T.ci[a], src[a]};
            std::sort(e.begin(), e.end());
            for (int32_t a = r0; a < r1; ++a) {
                T.ci[a] = e[(size_t)(a - r0)].first;
                src[a] = e[(size_t)(a - r0)].second;
            }
            continue;
        }
        for (int32_t a = r0 + 1; a < r1; ++a) {
            const int32_t c = T.ci[a], sk = src[a];
            int32_t b = a - 1;
            while (b >= r0 && T.ci[b] > c) {
                T.ci[b + 1] = T.ci[b];
                src[b + 1] = src[b];
                --b;
            }
            T.ci[b + 1] = c;
            src[b + 1] = sk;
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < nnz; ++p) {
        if (val) T.val[p] = val[src[p]];
        if (pos) (*pos)[src[p]] = (int32_t)p;
    }
}

// G^T of G = the pattern of tril(A) without a general transpose: where A's
// pattern is symmetric, row j of G^T holds the entries of A's row j with
// column >= j (ascending, as A's rows are).  pos[k] = position of G's entry
// k in it.  Returns false (T unusable) when some entry (i, j) of G has no
// (j, i) in A, i.e. the pattern is not symmetric; the caller then
// transposes.  Each G entry maps to a distinct position and both have the
// same count, so the map is the transpose's.
bool upper_transpose(const cg_handle *h, const int32_t *g_rp, const int32_t *g_ci, HostCsr &T,
                     HostArray<int32_t> &pos) {
    const int32_t n = h->n;
    const int32_t *arp = h->h_rp.data(), *aci = h->h_ci.data();
    T.rp.resize((size_t)n + 1);
    T.rp[0] = 0;   // the counts below write every other entry
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < n; ++j) {
        int32_t c = 0;
        for (int32_t k = arp[j]; k < arp[j + 1]; ++k) c += aci[k] >= j;
        T.rp[j + 1] = c;
    }
    par_running_sum(T.rp.data(), n);
    if (T.rp[n] != g_rp[n]) return false;
    T.ci.alloc((size_t)T.rp[n]);
    T.val.alloc(0);
    pos.alloc((size_t)g_rp[n]);
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < n; ++j) {
        int32_t p = T.rp[j];
        for (int32_t k = arp[j]; k < arp[j + 1]; ++k)
            if (aci[k] >= j) T.ci[p++] = aci[k];
    }
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = g_rp[i]; k < g_rp[i + 1]; ++k) {
            const int32_t j = g_ci[k];
            int32_t q = T.rp[j];
            while (q < T.rp[j + 1] && T.ci[q] < i) ++q;
            if (q < T.rp[j + 1] && T.ci[q] == i) pos[k] = q;
            else bad = 1;
        }
    return !bad;
}

// Upload G and G^T (schedules chosen automatically) and the work vectors;
// g_val null: the values are written on the device later.  pre: G^T's
// structure and the positions already built (then tpos is not written).
int install_factor(cg_handle *h, const int32_t *g_rp, const int32_t *g_ci, const double *g_val,
                   HostArray<int32_t> *tpos, const HostCsr *pre = nullptr) {
    HostCsr own;
    try {
        if (!pre) transpose(h->n, g_rp, g_ci, g_val, own, tpos);
    } catch (...) {
        return fail(CG_ENOMEM, "out of host memory");
    }
    const HostCsr &T = pre ? *pre : own;
    h->have_factor = false;
    // factors of cache-resident systems on 4 workgroups per CU (1024^2:
    // 43.2 against 43.8 us per PCG iteration with the automatic 8 per CU)
    const int fgrid = h->n <= (1 << 21) ? h->cus * 4 : 0;
    int rc = dm_upload(h->G, h->n, g_rp, g_ci, g_val, 0);
    if (!rc) rc = dm_schedule(h->G, 0, fgrid, h->cus, h->grid_cap, false);
    if (!rc) rc = dm_upload(h->GT, h->n, T.rp.data(), T.ci.data(), g_val ? T.val.data() : nullptr, 0);
    if (!rc) rc = dm_schedule(h->GT, 0, fgrid, h->cus, h->grid_cap, false);
    if (rc) return rc;
    if (!h->d_t) {
        hipError_t e = dmalloc(&h->d_t, (size_t)h->n + 2);
        if (e == hipSuccess) e = dmalloc(&h->d_z, (size_t)h->n + 2);
        if (e == hipSuccess) e = dmalloc(&h->d_r2, (size_t)h->n + 2);
        if (e != hipSuccess) return fail(CG_ENOMEM, "preconditioner vectors: %s", hipGetErrorString(e));
    }
    int32_t maxlen = 0;
    for (int32_t i = 0; i < h->n; ++i) maxlen = std::max(maxlen, g_rp[i + 1] - g_rp[i]);
    h->g_width = 0;
    for (int w = 1; w <= kFusedGWidth && !h->g_width; w <<= 1)
        if (maxlen <= w) h->g_width = w;
    return CG_OK;
}

int check_gpu_handle(const cg_handle *h) {
    if (!h) return fail(CG_EINVAL, "handle is NULL");
    if (!h->gpu_only()) return fail(CG_EINVAL, "the preconditioned solve needs a GPU-only handle");
    return CG_OK;
}

}  // namespace

namespace cgmi {

void fsai_free(cg_handle *h) {
    FsaiSetup *f = h->fsai;
    if (!f) return;
    (void)hipFree(f->d_scol);
    (void)hipFree(f->d_sval);
    (void)hipFree(f->d_diag);
    (void)hipFree(f->d_feats);
    (void)hipFree(f->d_err);
    (void)hipFree(f->d_theta);
    (void)hipFree(f->d_gpos);
    (void)hipFree(f->d_tpos);
    delete f;
    h->fsai = nullptr;
}

int solve_gpu_pcg(cg_handle *h, const double *b, double *x, double tol, int32_t maxit,
                  cg_result *res) {
    const int32_t n = h->n;
    hipStream_t st = h->stream;
    const int Ga = h->A.grid, Gg = h->G.grid, Gt = h->GT.grid, Gv = h->vec_grid;
    // the fused r/t kernel: one row per thread (CSR), or two 64-row slices per
    // wavefront (G in stencil slices; the grid a multiple of 8)
    const bool g_sten = h->G.sched.kind == kTileStencil && h->G.d_st_val;
    const int Gx = g_sten ? std::max(8, (int)std::min<int64_t>(h->grid_cap, ((((int64_t)n + 2 * kBlock - 1) / (2 * kBlock)) + 7) / 8 * 8))
                          : std::max(1, (int)std::min<int64_t>(h->grid_cap, ((int64_t)n + kBlock - 1) / kBlock));
    const Partials none = no_partials();
    const Partials setup_rr{h->d_part_setup, Ga}, setup_bb{h->d_part_setup + Ga, Ga};
    const Partials pq{h->d_part_pq, Ga}, rr{h->d_part_rr, h->g_width ? Gx : Gv}, rz{h->d_part_rz, Gt};
    if (fuse_dir_wanted(h, true) && h->g_width && !h->d_p2) {   // second p buffer of the fused direction update
        const hipError_t e = dmalloc(&h->d_p2, (size_t)h->n + 2);
        if (e != hipSuccess) return fail(CG_ENOMEM, "second p buffer: %s", hipGetErrorString(e));
    }
    HIP_TRY(hipMemcpyAsync(h->d_x, x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    int rc = gpu_state_init(h, tol, maxit);
    if (rc) return rc;
    double t_spmv = 0.0;
    int n_spmv = 0;
    const double t0 = now();
    // r = b - A x; z = G^T G r; rho_0 = r^T z; stop test; p = z
    HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, Ga, h->d_x, h->d_r, nullptr, b, h->d_p, h->d_part_setup,
                        none, none, nullptr, kSpmvResidual, 0, st));
    HIP_TRY(launch_spmv(h->G.dev(), h->G.sched, Gg, h->d_r, h->d_t, nullptr, nullptr, nullptr, nullptr,
                        none, none, nullptr, kSpmvPlain, 0, st));
    HIP_TRY(launch_spmv(h->GT.dev(), h->GT.sched, Gt, h->d_t, h->d_z, h->d_r, nullptr, nullptr,
                        h->d_part_rz, none, none, nullptr, kSpmvDot, 0, st));
    HIP_TRY(launch_update_p_pcg(n, Gv, h->d_z, h->d_p, nullptr, setup_rr, rz, setup_bb, h->d_state, 1, 0, st));
    const int C = h->opts.check_every;
    std::vector<hipEvent_t> ev;
    if (h->opts.profile) {
        ev.resize(2 * (size_t)C);
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    }
    const int P = h->opts.profile;   // events around the SpMV of every P-th iteration
    auto sampled = [P](int32_t it) { return P > 0 && it % P == 0; };
    double *const rbuf[2] = {h->d_r, h->d_r2};   // r of iterations k (even) and k (odd)
    // direction update fused into the next SpMV (x deferred, A in stencil
    // slices): p alternates between two buffers; the SpMV of iteration k+1
    // runs in the launch that ends iteration k (event slot j), iteration 0's
    // before the loop (the last slot pair)
    double *const pbuf[2] = {h->d_p, h->d_p2};
    const bool fused = h->g_width && h->d_p2 && fuse_dir_wanted(h, true) &&
                       spmv_dir_applies(h->A.dev(), h->A.sched, Ga, h->d_p, h->d_z, h->d_p2, h->d_x, h->d_q);
    if (fused && P) {
        ev.resize(2 * (size_t)C + 2);
        for (auto &e : ev)
            if (!e) HIP_TRY(hipEventCreate(&e));
    }
    bool first_pending = false;
    if (fused && maxit > 0) {
        first_pending = sampled(0);
        if (first_pending) HIP_TRY(hipEventRecord(ev[2 * (size_t)C], st));
        HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, Ga, pbuf[0], h->d_q, pbuf[0], nullptr, nullptr, h->d_part_pq,
                            none, none, h->d_state, kSpmvDot, 0, st));
        if (first_pending) HIP_TRY(hipEventRecord(ev[2 * (size_t)C + 1], st));
    }
    int32_t k = 0;
    bool running = maxit > 0;
    if (!running) rc = gpu_state_read(h);
    while (running) {
        const int32_t chunk = std::min<int32_t>(C, maxit - k);
        for (int32_t j = 0; j < chunk; ++j) {
            const int32_t kk = k + j;
            if (!fused) {
                if (sampled(kk)) HIP_TRY(hipEventRecord(ev[2 * j], st));
                HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, Ga, h->d_p, h->d_q, h->d_p, nullptr, nullptr,
                                    h->d_part_pq, none, none, h->d_state, kSpmvDot, 0, st));
                if (sampled(kk)) HIP_TRY(hipEventRecord(ev[2 * j + 1], st));
            }
            double *r_now = h->d_r;
            if (h->g_width) {
                // x/r update and t = G r in one kernel; r alternates between two buffers
                const double *r_old = rbuf[kk & 1];
                r_now = rbuf[(kk + 1) & 1];
                if (g_sten)
                    HIP_TRY(launch_pcg_xr_gs(n, Gx, h->G.d_st_off, h->G.d_st_offs, h->G.d_st_mask, h->G.d_st_val,
                                             r_old, r_now, h->d_q, h->d_t, h->d_part_rr, pq, h->d_state, kk, st));
                else
                    HIP_TRY(launch_pcg_xr_g(n, Gx, h->g_width, h->G.d_rp, h->G.d_ci, h->G.d_val, r_old, r_now,
                                            h->d_q, h->d_t, h->d_part_rr, pq, h->d_state, kk, st));
            } else {
                HIP_TRY(launch_update_xr(n, Gv, h->d_x, h->d_r, h->d_p, h->d_q, h->d_part_rr, pq, h->d_state, 1,
                                         kk, 0.0, st));
                HIP_TRY(launch_spmv(h->G.dev(), h->G.sched, Gg, h->d_r, h->d_t, nullptr, nullptr, nullptr,
                                    nullptr, none, none, h->d_state, kSpmvPlain, 0, st));
            }
            HIP_TRY(launch_spmv(h->GT.dev(), h->GT.sched, Gt, h->d_t, h->d_z, r_now, nullptr, nullptr,
                                h->d_part_rz, none, none, h->d_state, kSpmvDot, 0, st));
            if (fused) {
                if (sampled(kk + 1)) HIP_TRY(hipEventRecord(ev[2 * j], st));
                HIP_TRY(launch_spmv_dir(h->A.dev(), h->A.sched, Ga, pbuf[kk & 1], h->d_z, pbuf[(kk + 1) & 1],
                                        h->d_x, h->d_q, h->d_part_pq, rr, rz, h->d_state, kk, 1, st));
                if (sampled(kk + 1)) HIP_TRY(hipEventRecord(ev[2 * j + 1], st));
            } else {
                // x += alpha p here when the fused kernel formed r (it leaves x alone)
                HIP_TRY(launch_update_p_pcg(n, Gv, h->d_z, h->d_p, h->g_width ? h->d_x : nullptr, rr, rz, none,
                                            h->d_state, 0, kk, st));
            }
        }
        const int32_t it0 = k;
        k += chunk;
        rc = gpu_state_read(h);
        if (rc) break;
        running = h->h_state->done == kDoneRunning && k < maxit;
        if (fused && P) {
            const DevState &s = *h->h_state;
            float ms = 0.f;
            if (first_pending) {
                first_pending = false;
                if (fused_spmv_ran(s, 0)) {
                    HIP_TRY(hipEventElapsedTime(&ms, ev[2 * (size_t)C], ev[2 * (size_t)C + 1]));
                    t_spmv += 1e-3 * ms;
                    ++n_spmv;
                }
            }
            for (int32_t j = 0; j < chunk; ++j) {
                const int32_t i = it0 + j + 1;
                if (!sampled(i) || !fused_spmv_ran(s, i)) continue;
                HIP_TRY(hipEventElapsedTime(&ms, ev[2 * j], ev[2 * j + 1]));
                t_spmv += 1e-3 * ms;
                ++n_spmv;
            }
        } else if (h->opts.profile) {
            int32_t ran = h->h_state->iter - it0 + (h->h_state->done == kDoneBreakdown ? 1 : 0);
            ran = std::max(0, std::min<int32_t>(ran, chunk));
            for (int32_t j = 0; j < ran; ++j) {
                if (!sampled(it0 + j)) continue;
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev[2 * j], ev[2 * j + 1]));
                t_spmv += 1e-3 * ms;
                ++n_spmv;
            }
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (rc) return rc;
    const double t_gpu = now() - t0;
    const DevState s = *h->h_state;
    if (s.bb == 0.0) {  // b = 0: the solution is x = 0
        HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * n, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (res) {
            res->status = CG_OK;
            res->converged = 1;
        }
        return CG_OK;
    }
    if (s.done == kDoneBreakdown) {
        // x is left as given: the caller restarts without the preconditioner
        if (res) {
            res->status = CG_EBREAKDOWN;
            res->iterations = s.iter;
            res->t_gpu = t_gpu;
        }
        return CG_EBREAKDOWN;
    }
    HIP_TRY(hipMemcpyAsync(x, h->d_x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    double rr_true = 0.0, bb = 0.0;
    rc = gpu_true_residual(h, b, x, &rr_true, &bb);
    if (rc) return rc;
    const int status = status_of(s.done == kDoneRunning ? kDoneMaxit : s.done);
    if (res) {
        res->status = status;
        res->iterations = s.iter;
        res->converged = status == CG_OK;
        res->rel_res_recur = std::sqrt(s.rr) / std::sqrt(s.bb);
        res->rel_res_true = std::sqrt(rr_true) / std::sqrt(bb);
        res->t_gpu = t_gpu;
        res->t_spmv = t_spmv;
        res->n_spmv = n_spmv;
        res->fused_dir = fused;
    }
    return status;
}

}  // namespace cgmi

// ---------------------------------------------------------------------------
// factor installation

extern "C" int cg_set_fsai(cg_handle *h, int64_t nnz, const int32_t *g_row_ptr, const int32_t *g_col,
                           const double *g_val) {
    clear_error();
    int rc = check_gpu_handle(h);
    if (rc) return rc;
    rc = validate_csr(h->n, nnz, g_row_ptr, g_col, g_val);
    if (rc) return rc;
    if (nnz == 0) return fail(CG_EINVAL, "the factor has no nonzeros");
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(h->stream ? hipStreamSynchronize(h->stream) : hipDeviceSynchronize());
    fsai_free(h);
    rc = install_factor(h, g_row_ptr, g_col, g_val, nullptr);
    if (rc) return rc;
    h->have_factor = true;
    return CG_OK;
}

// Classic FSAI: per row, the Cholesky factor L of the local block
// M = A[P, P] (columns of tril(A) row i, i last), then g = M^-1 e_last by
// the two triangular solves; g_last = 1 / L_last,last^2, so the scaled row
// g / sqrt(g_last) is g * L_last,last.
extern "C" int cg_fsai_classic(cg_handle *h) {
    clear_error();
    int rc = check_gpu_handle(h);
    if (rc) return rc;
    const int32_t n = h->n;
    constexpr int kMax = CG_FSAI_CLASSIC_MAX_ROW;
    std::vector<int32_t> g_rp, g_ci;
    std::vector<double> g_val;
    try {
        g_rp.assign((size_t)n + 1, 0);
        int32_t bad_row = INT32_MAX, bad_kind = 0;
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            int cnt = 0;
            bool diag = false;
            for (int32_t k = h->h_rp[i]; k < h->h_rp[i + 1] && h->h_ci[k] <= i; ++k) {
                ++cnt;
                diag = h->h_ci[k] == i;
            }
            g_rp[i + 1] = cnt;
            const int kind = !diag ? 1 : cnt > kMax ? 2 : 0;
            if (kind) {
#pragma omp critical(cgmi_classic_bad_row)
                if (i < bad_row) {
                    bad_row = i;
                    bad_kind = kind;
                }
            }
        }
        if (bad_kind == 1) return fail(CG_EINVAL, "row %d has no diagonal entry", bad_row);
        if (bad_kind == 2)
            return fail(CG_EINVAL, "row %d of tril(A) has more than %d entries", bad_row, kMax);
        par_running_sum(g_rp.data(), n);
        g_ci.resize((size_t)g_rp[n]);
        g_val.resize((size_t)g_rp[n]);
        bad_row = INT32_MAX;
        // entry (r, c) of A by a scan of row r (columns ascending)
        auto a_at = [&](int32_t r, int32_t c) {
            for (int32_t k = h->h_rp[r]; k < h->h_rp[r + 1] && h->h_ci[k] <= c; ++k)
                if (h->h_ci[k] == c) return h->h_val[k];
            return 0.0;
        };
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            const int32_t b = g_rp[i];
            const int m = g_rp[i + 1] - b;
            int32_t P[kMax];
            for (int e = 0; e < m; ++e) P[e] = g_ci[(size_t)b + e] = h->h_ci[h->h_rp[i] + e];
            double L[kMax][kMax] = {};
            bool ok = true;
            for (int c = 0; c < m && ok; ++c) {
                for (int r = c; r < m; ++r) {
                    double v = a_at(P[r], P[c]);
                    for (int k = 0; k < c; ++k) v -= L[r][k] * L[c][k];
                    if (r == c) {
                        if (!(v > 0.0)) {
                            ok = false;
                            break;
                        }
                        L[c][c] = std::sqrt(v);
                    } else {
                        L[r][c] = v / L[c][c];
                    }
                }
            }
            if (!ok) {
#pragma omp critical(cgmi_classic_bad_row)
                bad_row = std::min(bad_row, i);
                continue;
            }
            double g[kMax];
            g[m - 1] = 1.0 / (L[m - 1][m - 1] * L[m - 1][m - 1]);
            for (int r = m - 2; r >= 0; --r) {
                double v = 0.0;
                for (int j = r + 1; j < m; ++j) v -= L[j][r] * g[j];
                g[r] = v / L[r][r];
            }
            for (int e = 0; e < m; ++e) g_val[(size_t)b + e] = g[e] * L[m - 1][m - 1];
        }
        if (bad_row != INT32_MAX)
            return fail(CG_EINVAL, "the local system of row %d is not positive definite", bad_row);
    } catch (...) {
        return fail(CG_ENOMEM, "out of host memory");
    }
    return cg_set_fsai(h, (int64_t)g_rp[n], g_rp.data(), g_ci.data(), g_val.data());
}

namespace {

// Structure of the learned factor: G on the pattern of tril(A) and the
// positions of each row's C, W, S entries.
int build_learned_structure(cg_handle *h) {
    const int32_t n = h->n;
    HostVec<int32_t> g_rp;
    HostArray<int32_t> g_ci, gpos, tpos;
    try {
        g_rp.resize((size_t)n + 1);
        g_rp[0] = 0;   // pass 1 writes every other entry
        gpos.alloc((size_t)n * 3);
        // pass 1 (rows in parallel): check the stencil, count tril entries;
        // the first offending row is reported
        int32_t bad_row = INT32_MAX, bad_kind = 0;
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            int seen[kSlots] = {0, 0, 0, 0, 0};
            int kind = 0, cnt = 0;
            for (int32_t k = h->h_rp[i]; k < h->h_rp[i + 1]; ++k) {
                const int s = stencil_slot(i, h->h_ci[k]);
                if (seen[s]++) kind = 1;
                if (h->h_ci[k] > i) continue;
                if (s == kSlotC && !(h->h_val[k] > 0.0)) kind = kind ? kind : 2;
                ++cnt;
            }
            if (!seen[kSlotC] && !kind) kind = 3;
            g_rp[i + 1] = cnt;
            if (kind) {
#pragma omp critical(cgmi_fsai_bad_row)
                if (i < bad_row) {
                    bad_row = i;
                    bad_kind = kind;
                }
            }
        }
        if (bad_kind == 1) return fail(CG_EINVAL, "row %d is not a 5-point stencil row", bad_row);
        if (bad_kind == 2) return fail(CG_EINVAL, "diagonal of row %d is not positive", bad_row);
        if (bad_kind == 3) return fail(CG_EINVAL, "row %d has no diagonal entry", bad_row);
        par_running_sum(g_rp.data(), n);
        g_ci.alloc((size_t)g_rp[n]);
        // pass 2: columns and slot positions (-1: no such neighbour)
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            gpos[(size_t)i * 3] = gpos[(size_t)i * 3 + 1] = gpos[(size_t)i * 3 + 2] = -1;
            int32_t p = g_rp[i];
            for (int32_t k = h->h_rp[i]; k < h->h_rp[i + 1]; ++k) {
                if (h->h_ci[k] > i) continue;
                const int s = stencil_slot(i, h->h_ci[k]);
                const int m = s == kSlotC ? 0 : s == kSlotW ? 1 : 2;
                gpos[(size_t)i * 3 + m] = p;
                g_ci[p++] = h->h_ci[k];
            }
        }
    } catch (...) {
        return fail(CG_ENOMEM, "out of host memory");
    }
    // G^T from A's upper triangle where A's pattern is symmetric, else by transposing G
    HostCsr T;
    bool direct = false;
    try {
        direct = upper_transpose(h, g_rp.data(), g_ci.data(), T, tpos);
    } catch (...) {
        return fail(CG_ENOMEM, "out of host memory");
    }
    int rc = install_factor(h, g_rp.data(), g_ci.data(), nullptr, &tpos, direct ? &T : nullptr);   // values come from the device
    if (rc) return rc;
    FsaiSetup *f = new (std::nothrow) FsaiSetup();
    if (!f) return fail(CG_ENOMEM, "out of host memory");
    h->fsai = f;
    const size_t nn = (size_t)n;
    hipError_t e = dmalloc(&f->d_scol, nn * kSlots);
    if (e == hipSuccess) e = dmalloc(&f->d_sval, nn * kSlots);
    if (e == hipSuccess) e = dmalloc(&f->d_diag, nn);
    if (e == hipSuccess) e = dmalloc(&f->d_feats, nn * kFeatPad);
    if (e == hipSuccess) e = dmalloc(&f->d_err, 1);
    if (e == hipSuccess) e = dmalloc(&f->d_theta, kNParams);
    if (e == hipSuccess) e = dmalloc(&f->d_gpos, nn * 3);
    if (e == hipSuccess) e = dmalloc(&f->d_tpos, tpos.size());
    if (e != hipSuccess) return fail(CG_ENOMEM, "learned-factor workspace: %s", hipGetErrorString(e));
    hipStream_t st = h->stream;
    HIP_TRY(hipMemcpy(f->d_gpos, gpos.data(), sizeof(int32_t) * gpos.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(f->d_tpos, tpos.data(), sizeof(int32_t) * tpos.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemsetAsync(f->d_err, 0, sizeof(int32_t), st));
    HIP_TRY(hipMemsetAsync(f->d_feats, 0, sizeof(uint16_t) * nn * kFeatPad, st));
    HIP_TRY(fsai_prepare(n, h->A.d_rp, h->A.d_ci, h->A.d_val, f->d_scol, f->d_sval, f->d_diag, f->d_feats,
                         f->d_err, st));
    int32_t bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, f->d_err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) return fail(CG_EINVAL, "%d rows are not 5-point rows with positive diagonals", bad);
    return CG_OK;
}

}  // namespace

extern "C" int cg_fsai_setup(cg_handle *h, const float *theta) {
    clear_error();
    int rc = check_gpu_handle(h);
    if (rc) return rc;
    if (!theta) return fail(CG_EINVAL, "theta is NULL");
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(h->stream ? hipStreamSynchronize(h->stream) : hipDeviceSynchronize());
    if (!h->fsai) {
        rc = build_learned_structure(h);
        if (rc) {
            fsai_free(h);
            h->have_factor = false;
            return rc;
        }
    }
    FsaiSetup *f = h->fsai;
    hipStream_t st = h->stream;
    h->have_factor = false;
    HIP_TRY(hipMemcpyAsync(f->d_theta, theta, sizeof(float) * kNParams, hipMemcpyHostToDevice, st));
    HIP_TRY(fsai_forward_factor(h->n, f->d_feats, f->d_theta, f->d_scol, f->d_diag, f->d_gpos, f->d_tpos,
                                h->G.d_val, h->GT.d_val, st));
    for (DevMatrix *M : {&h->G, &h->GT}) {
        if (M->sched.kind == kTileSliced || M->sched.kind == kTileSlicedDict)
            HIP_TRY(sell_refresh(M->m, M->sched.ntiles, M->d_rp, M->d_sell_off, M->d_val, M->d_sell_val, st));
        if (M->sched.kind == kTileStencil)
            HIP_TRY(stencil_refresh(M->m, (M->m + 63) / 64, M->d_rp, M->d_st_off, M->d_st_mask, M->d_val,
                                    M->d_st_val, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    h->have_factor = true;
    return CG_OK;
}

extern "C" int cg_fsai_factor_info(const cg_handle *h, int64_t *nnz) {
    clear_error();
    if (!h || !nnz) return fail(CG_EINVAL, "NULL argument");
    if (!h->have_factor) return fail(CG_EINVAL, "no factor installed");
    *nnz = h->G.nnz;
    return CG_OK;
}

extern "C" int cg_fsai_read_factor(const cg_handle *h, int32_t *g_row_ptr, int32_t *g_col, double *g_val) {
    clear_error();
    if (!h) return fail(CG_EINVAL, "handle is NULL");
    if (!h->have_factor) return fail(CG_EINVAL, "no factor installed");
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(h->stream ? hipStreamSynchronize(h->stream) : hipDeviceSynchronize());
    const size_t nnz = (size_t)h->G.nnz;
    if (g_row_ptr) std::memcpy(g_row_ptr, h->G.h_rp.data(), sizeof(int32_t) * ((size_t)h->n + 1));
    if (g_col) std::memcpy(g_col, h->G.h_ci.data(), sizeof(int32_t) * nnz);
    if (g_val) HIP_TRY(hipMemcpy(g_val, h->G.d_val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    return CG_OK;
}

// ---------------------------------------------------------------------------
// training

struct cg_fsai_trainer {
    int dev = 0;
    hipStream_t stream = nullptr;
    int32_t nsys = 0;
    std::vector<int32_t> n;
    std::vector<int64_t> base;   // first row of each system (a multiple of 16)
    int64_t rows = 0;            // rows incl. padding
    int32_t *d_scol = nullptr;
    float *d_sval = nullptr;
    double *d_diag = nullptr;
    uint16_t *d_feats = nullptr;
    float *d_out = nullptr;
    int64_t *d_dg = nullptr;     // dL/dG~ in 64-bit fixed point (rows x 3)
    float *d_theta = nullptr, *d_m = nullptr, *d_v = nullptr, *d_theta_eval = nullptr, *d_grad = nullptr;
    float *d_gpart = nullptr;
    double *d_lpart = nullptr;
    size_t lpart_cap = 0;
    uint8_t *d_stage = nullptr;  // a step's tile list and samples, uploaded in one copy
    size_t stage_cap = 0;
    int32_t step = 0;
};

namespace {

constexpr int kTrainGrid = 256;   // workgroups of the backward pass (gradient partials)

void trainer_free(cg_fsai_trainer *t) {
    for (void *p : {(void *)t->d_scol, (void *)t->d_sval, (void *)t->d_diag, (void *)t->d_feats,
                    (void *)t->d_out, (void *)t->d_dg, (void *)t->d_theta, (void *)t->d_m,
                    (void *)t->d_v, (void *)t->d_theta_eval, (void *)t->d_grad, (void *)t->d_gpart,
                    (void *)t->d_lpart, (void *)t->d_stage})
        (void)hipFree(p);
    delete t;
}

template <class T>
int ensure_capacity(T **p, size_t &cap, size_t need) {
    if (need <= cap && *p) return CG_OK;
    (void)hipFree(*p);
    *p = nullptr;
    cap = 0;
    const hipError_t e = dmalloc(p, need);
    if (e != hipSuccess) return fail(CG_ENOMEM, "trainer buffers: %s", hipGetErrorString(e));
    cap = need;
    return CG_OK;
}

// Forward, loss, backward and (adam_step >= 1) an Adam step, or the gradient
// only (adam_step = 0), on the sampled rows.
int run_loss_grad(cg_fsai_trainer *t, const float *theta, int32_t nsel, const int32_t *sys,
                  int32_t rows_per_sys, const int32_t *rows, int32_t adam_step, double lr, double *loss,
                  float *grad_host) {
    if (nsel <= 0 || rows_per_sys <= 0) return fail(CG_EINVAL, "nsel and rows_per_sys must be >= 1");
    if (!sys || !rows) return fail(CG_EINVAL, "sys/rows is NULL");
    const int64_t nsamp64 = (int64_t)nsel * rows_per_sys;
    if (nsamp64 > INT32_MAX / 2) return fail(CG_EINVAL, "too many samples");
    const int32_t nsamp = (int32_t)nsamp64;
    for (int32_t s = 0; s < nsel; ++s) {
        if (sys[s] < 0 || sys[s] >= t->nsys) return fail(CG_EINVAL, "system %d out of range", sys[s]);
        for (int32_t r = 0; r < rows_per_sys; ++r) {
            const int32_t row = rows[(size_t)s * rows_per_sys + r];
            if (row < 0 || row >= t->n[sys[s]])
                return fail(CG_EINVAL, "row %d out of range for system %d", row, sys[s]);
        }
    }
    std::vector<int32_t> uniq(sys, sys + nsel);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    int64_t ntiles64 = 0;
    for (int32_t s : uniq) ntiles64 += (t->n[s] + 15) / 16;
    if (ntiles64 > INT32_MAX / 4) return fail(CG_EINVAL, "too many rows in one step");
    const int32_t ntiles = (int32_t)ntiles64;
    // staging: tiles (int32), sample rows (int32), system sizes (int32),
    // system first rows (int64), each at an 8-byte aligned offset
    auto up8 = [](size_t b) { return (b + 7) & ~(size_t)7; };
    const size_t o_srow = up8(sizeof(int32_t) * (size_t)ntiles);
    const size_t o_sn = up8(o_srow + sizeof(int32_t) * (size_t)nsamp);
    const size_t o_sbase = up8(o_sn + sizeof(int32_t) * (size_t)nsamp);
    const size_t bytes = o_sbase + sizeof(int64_t) * (size_t)nsamp;
    std::vector<uint8_t> blob(bytes, 0);
    int32_t *tiles = reinterpret_cast<int32_t *>(blob.data());
    int32_t *srow = reinterpret_cast<int32_t *>(blob.data() + o_srow);
    int32_t *sn = reinterpret_cast<int32_t *>(blob.data() + o_sn);
    int64_t *sbase = reinterpret_cast<int64_t *>(blob.data() + o_sbase);
    int32_t nt = 0;
    for (int32_t s : uniq)
        for (int64_t r = 0; r < t->n[s]; r += 16) tiles[nt++] = (int32_t)(t->base[s] + r);
    for (int32_t k = 0; k < nsamp; ++k) {
        const int32_t s = sys[k / rows_per_sys];
        srow[k] = rows[k];
        sbase[k] = t->base[s];
        sn[k] = t->n[s];
    }
    const int32_t lblocks = fsai_loss_blocks(nsamp);
    int rc = ensure_capacity(&t->d_stage, t->stage_cap, bytes);
    if (!rc) rc = ensure_capacity(&t->d_lpart, t->lpart_cap, (size_t)lblocks);
    if (rc) return rc;
    const int32_t *d_tiles = reinterpret_cast<const int32_t *>(t->d_stage);
    const int32_t *d_srow = reinterpret_cast<const int32_t *>(t->d_stage + o_srow);
    const int32_t *d_sn = reinterpret_cast<const int32_t *>(t->d_stage + o_sn);
    const int64_t *d_sbase = reinterpret_cast<const int64_t *>(t->d_stage + o_sbase);
    hipStream_t st = t->stream;
    HIP_TRY(hipMemcpyAsync(t->d_stage, blob.data(), bytes, hipMemcpyHostToDevice, st));
    // outputs of every row of the sampled systems, their dL/dG~ cleared
    HIP_TRY(fsai_forward_outputs(ntiles, d_tiles, t->rows, t->d_feats, theta, t->d_out, t->d_dg, st));
    HIP_TRY(fsai_loss(nsamp, d_srow, d_sbase, d_sn, t->d_out, t->d_scol, t->d_sval, t->d_dg,
                      (float)(2.0 / nsamp), t->d_lpart, st));
    const int32_t grid = std::max(1, std::min(kTrainGrid, (ntiles + 3) / 4));
    HIP_TRY(fsai_backward(ntiles, d_tiles, t->d_feats, theta, t->d_out, t->d_dg, t->d_scol, t->d_gpart, grid,
                          st));
    HIP_TRY(fsai_adam(grid, t->d_gpart, t->d_theta, t->d_m, t->d_v, t->d_grad, adam_step, (float)lr, st));
    std::vector<double> lp((size_t)lblocks);
    HIP_TRY(hipMemcpyAsync(lp.data(), t->d_lpart, sizeof(double) * lblocks, hipMemcpyDeviceToHost, st));
    if (grad_host) HIP_TRY(hipMemcpyAsync(grad_host, t->d_grad, sizeof(float) * kNParams, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double sum = 0.0;
    for (double v : lp) sum += v;
    if (loss) *loss = sum / nsamp;
    return CG_OK;
}

}  // namespace

extern "C" int cg_fsai_trainer_create(int32_t nsys, const int32_t *n, const int64_t *nnz,
                                      const int32_t *const *row_ptr, const int32_t *const *col,
                                      const double *const *val, const float *theta0,
                                      cg_fsai_trainer **out) {
    clear_error();
    if (!out) return fail(CG_EINVAL, "out is NULL");
    *out = nullptr;
    if (nsys <= 0) return fail(CG_EINVAL, "nsys must be >= 1");
    if (!n || !nnz || !row_ptr || !col || !val || !theta0) return fail(CG_EINVAL, "NULL argument");
    int64_t rows = 0, max_nnz = 0;
    int32_t max_n = 0;
    for (int32_t s = 0; s < nsys; ++s) {
        if (n[s] <= 0) return fail(CG_EINVAL, "system %d is empty", s);
        const int rc = validate_csr(n[s], nnz[s], row_ptr[s], col[s], val[s]);
        if (rc) return rc;
        rows += ((int64_t)n[s] + 15) / 16 * 16;
        max_n = std::max(max_n, n[s]);
        max_nnz = std::max(max_nnz, nnz[s]);
    }
    if (rows > INT32_MAX / kSlots) return fail(CG_EINVAL, "training set too large");
    cg_fsai_trainer *t = new (std::nothrow) cg_fsai_trainer();
    if (!t) return fail(CG_ENOMEM, "out of host memory");
    auto bail = [&](int code) {
        trainer_free(t);
        return code;
    };
    if (hipGetDevice(&t->dev) != hipSuccess) return bail(fail(CG_EDEVICE, "no HIP device"));
    t->nsys = nsys;
    t->rows = rows;
    try {
        t->n.assign(n, n + nsys);
        t->base.resize(nsys);
    } catch (...) {
        return bail(fail(CG_ENOMEM, "out of host memory"));
    }
    int64_t b = 0;
    for (int32_t s = 0; s < nsys; ++s) {
        t->base[s] = b;
        b += ((int64_t)n[s] + 15) / 16 * 16;
    }
    const size_t R = (size_t)rows;
    hipError_t e = dmalloc(&t->d_scol, R * kSlots);
    if (e == hipSuccess) e = dmalloc(&t->d_sval, R * kSlots);
    if (e == hipSuccess) e = dmalloc(&t->d_diag, R);
    if (e == hipSuccess) e = dmalloc(&t->d_feats, R * kFeatPad);
    if (e == hipSuccess) e = dmalloc(&t->d_out, R * kOutPad);
    if (e == hipSuccess) e = dmalloc(&t->d_dg, R * 3);
    if (e == hipSuccess) e = dmalloc(&t->d_theta, kNParams);
    if (e == hipSuccess) e = dmalloc(&t->d_m, kNParams);
    if (e == hipSuccess) e = dmalloc(&t->d_v, kNParams);
    if (e == hipSuccess) e = dmalloc(&t->d_theta_eval, kNParams);
    if (e == hipSuccess) e = dmalloc(&t->d_grad, kNParams);
    if (e == hipSuccess) e = dmalloc(&t->d_gpart, (size_t)kTrainGrid * kNParams);
    if (e != hipSuccess) return bail(fail(CG_ENOMEM, "trainer allocation: %s", hipGetErrorString(e)));
    // padding rows: no features and no slots (their dL/dG~ is cleared with
    // the other rows of their tiles at every step)
    if (e == hipSuccess) e = hipMemset(t->d_feats, 0, sizeof(uint16_t) * R * kFeatPad);
    if (e == hipSuccess) e = hipMemset(t->d_scol, 0xFF, sizeof(int32_t) * R * kSlots);
    if (e == hipSuccess) e = hipMemset(t->d_m, 0, sizeof(float) * kNParams);
    if (e == hipSuccess) e = hipMemset(t->d_v, 0, sizeof(float) * kNParams);
    if (e == hipSuccess) e = hipMemcpy(t->d_theta, theta0, sizeof(float) * kNParams, hipMemcpyHostToDevice);
    // features of each system from its own (local-index) CSR
    int32_t *d_rp = nullptr, *d_ci = nullptr, *d_err = nullptr;
    double *d_val = nullptr;
    if (e == hipSuccess) e = dmalloc(&d_rp, (size_t)max_n + 1);
    if (e == hipSuccess) e = dmalloc(&d_ci, (size_t)max_nnz);
    if (e == hipSuccess) e = dmalloc(&d_val, (size_t)max_nnz);
    if (e == hipSuccess) e = dmalloc(&d_err, 1);
    if (e == hipSuccess) e = hipMemset(d_err, 0, sizeof(int32_t));
    for (int32_t s = 0; s < nsys && e == hipSuccess; ++s) {
        e = hipMemcpy(d_rp, row_ptr[s], sizeof(int32_t) * ((size_t)n[s] + 1), hipMemcpyHostToDevice);
        if (e == hipSuccess && nnz[s])
            e = hipMemcpy(d_ci, col[s], sizeof(int32_t) * (size_t)nnz[s], hipMemcpyHostToDevice);
        if (e == hipSuccess && nnz[s])
            e = hipMemcpy(d_val, val[s], sizeof(double) * (size_t)nnz[s], hipMemcpyHostToDevice);
        const size_t o = (size_t)t->base[s];
        if (e == hipSuccess)
            e = fsai_prepare(n[s], d_rp, d_ci, d_val, t->d_scol + o * kSlots, t->d_sval + o * kSlots,
                             t->d_diag + o, t->d_feats + o * kFeatPad, d_err, t->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
    }
    int32_t bad = 0;
    if (e == hipSuccess) e = hipMemcpy(&bad, d_err, sizeof(int32_t), hipMemcpyDeviceToHost);
    (void)hipFree(d_rp);
    (void)hipFree(d_ci);
    (void)hipFree(d_val);
    (void)hipFree(d_err);
    if (e != hipSuccess) return bail(fail(CG_EDEVICE, "trainer setup: %s", hipGetErrorString(e)));
    if (bad) return bail(fail(CG_EINVAL, "%d rows are not 5-point rows with positive diagonals", bad));
    *out = t;
    return CG_OK;
}

extern "C" void cg_fsai_trainer_destroy(cg_fsai_trainer *t) {
    if (!t) return;
    (void)hipSetDevice(t->dev);
    (void)hipDeviceSynchronize();
    trainer_free(t);
}

extern "C" int cg_fsai_loss_grad(cg_fsai_trainer *t, const float *theta, int32_t nsel, const int32_t *sys,
                                 int32_t rows_per_sys, const int32_t *rows, double *loss, float *grad,
                                 float *outputs) {
    clear_error();
    if (!t) return fail(CG_EINVAL, "trainer is NULL");
    HIP_TRY(hipSetDevice(t->dev));
    const float *th = t->d_theta;
    if (theta) {
        HIP_TRY(hipMemcpy(t->d_theta_eval, theta, sizeof(float) * kNParams, hipMemcpyHostToDevice));
        th = t->d_theta_eval;
    }
    int rc = run_loss_grad(t, th, nsel, sys, rows_per_sys, rows, 0, 0.0, loss, grad);
    if (rc) return rc;
    if (outputs) {
        const int32_t s = sys[0];
        HIP_TRY(hipMemcpy2D(outputs, sizeof(float) * kOut, t->d_out + t->base[s] * kOutPad,
                            sizeof(float) * kOutPad, sizeof(float) * kOut, (size_t)t->n[s],
                            hipMemcpyDeviceToHost));
    }
    return CG_OK;
}

extern "C" int cg_fsai_train_step(cg_fsai_trainer *t, int32_t nsel, const int32_t *sys, int32_t rows_per_sys,
                                  const int32_t *rows, double lr, double *loss) {
    clear_error();
    if (!t) return fail(CG_EINVAL, "trainer is NULL");
    if (!(lr > 0.0) || !std::isfinite(lr)) return fail(CG_EINVAL, "lr must be positive");
    HIP_TRY(hipSetDevice(t->dev));
    const int rc = run_loss_grad(t, t->d_theta, nsel, sys, rows_per_sys, rows, t->step + 1, lr, loss, nullptr);
    if (rc) return rc;
    ++t->step;
    return CG_OK;
}

extern "C" int cg_fsai_get_params(const cg_fsai_trainer *t, float *theta) {
    clear_error();
    if (!t || !theta) return fail(CG_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(t->dev));
    HIP_TRY(hipMemcpy(theta, t->d_theta, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
    return CG_OK;
}

extern "C" int cg_fsai_get_state(const cg_fsai_trainer *t, float *theta, float *m, float *v, int32_t *step) {
    clear_error();
    if (!t) return fail(CG_EINVAL, "NULL trainer");
    HIP_TRY(hipSetDevice(t->dev));
    if (t->stream) HIP_TRY(hipStreamSynchronize(t->stream));
    if (theta) HIP_TRY(hipMemcpy(theta, t->d_theta, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
    if (m) HIP_TRY(hipMemcpy(m, t->d_m, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
    if (v) HIP_TRY(hipMemcpy(v, t->d_v, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
    if (step) *step = t->step;
    return CG_OK;
}

extern "C" int cg_fsai_set_state(cg_fsai_trainer *t, const float *theta, const float *m, const float *v,
                                 int32_t step) {
    clear_error();
    if (!t) return fail(CG_EINVAL, "NULL trainer");
    if (step < 0) return fail(CG_EINVAL, "step must be >= 0");
    HIP_TRY(hipSetDevice(t->dev));
    if (t->stream) HIP_TRY(hipStreamSynchronize(t->stream));
    if (theta) HIP_TRY(hipMemcpy(t->d_theta, theta, sizeof(float) * kNParams, hipMemcpyHostToDevice));
    if (m) HIP_TRY(hipMemcpy(t->d_m, m, sizeof(float) * kNParams, hipMemcpyHostToDevice));
    if (v) HIP_TRY(hipMemcpy(t->d_v, v, sizeof(float) * kNParams, hipMemcpyHostToDevice));
    t->step = step;
    return CG_OK;
}

extern "C" int cg_fsai_features(const cg_fsai_trainer *t, int32_t sys, float *feats) {
    clear_error();
    if (!t || !feats) return fail(CG_EINVAL, "NULL argument");
    if (sys < 0 || sys >= t->nsys) return fail(CG_EINVAL, "system %d out of range", sys);
    HIP_TRY(hipSetDevice(t->dev));
    const size_t n = (size_t)t->n[sys];
    std::vector<uint16_t> raw(n * kFeatPad);
    HIP_TRY(hipMemcpy(raw.data(), t->d_feats + (size_t)t->base[sys] * kFeatPad, sizeof(uint16_t) * raw.size(),
                      hipMemcpyDeviceToHost));
    for (size_t i = 0; i < n; ++i)
        for (int k = 0; k < kFeat; ++k) {
            const uint32_t u = (uint32_t)raw[i * kFeatPad + k] << 16;
            float f;
            std::memcpy(&f, &u, sizeof f);
            feats[i * kFeat + k] = f;
        }
    return CG_OK;
}
