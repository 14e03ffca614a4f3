// batch.cpp -- host side of the batched persistent solve: stacking of the
// systems, team assignment from the schedule, the cooperative launch and the
// per-pair results.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdlib>
#include <new>
#include <vector>

#include "../../include/cgmi_batch.h"
#include "batch_internal.h"
#include "cgmi_host.h"

using namespace cgmi;

#define HIP_TRY(expr) CGMI_HIP_TRY(expr)

struct cg_batch {
    int dev = 0;
    hipStream_t stream = nullptr;
    int32_t nsys = 0, nrhs = 0;
    int64_t n_total = 0, nnz_total = 0;
    std::vector<int64_t> row_off;   // nsys + 1
    int cus = 256;
    cg_batch_sched sched{};
    // device
    int32_t *d_rp = nullptr, *d_ci = nullptr;
    double *d_val = nullptr;
    double *d_R = nullptr, *d_P = nullptr, *d_Q = nullptr;
    double *d_part = nullptr;
    int32_t *d_bar = nullptr, *d_err = nullptr, *d_episodes = nullptr;
    int32_t *d_wg_item = nullptr, *d_item_sys = nullptr, *d_item_rank = nullptr;
    int32_t *d_team_first = nullptr, *d_team_size = nullptr;
    int64_t item_cap = 0;       // entries of d_item_sys / d_item_rank
    int64_t *d_row_off = nullptr;
    int32_t *d_strip = nullptr;      // [nsys] line length of a strip-ordered phase A (0: row order)
    BatchOutDev *d_out = nullptr;
    int grid_cap = 0;                // workgroups the buffers are sized for
    // current team assignment
    int grid = 0;
    std::vector<int32_t> team_size;
};

namespace {

void batch_free(cg_batch *b) {
    for (void *p : {(void *)b->d_rp, (void *)b->d_ci, (void *)b->d_val, (void *)b->d_R, (void *)b->d_P,
                    (void *)b->d_Q, (void *)b->d_part, (void *)b->d_bar, (void *)b->d_err,
                    (void *)b->d_episodes, (void *)b->d_wg_item, (void *)b->d_item_sys, (void *)b->d_item_rank,
                    (void *)b->d_team_first, (void *)b->d_team_size, (void *)b->d_row_off,
                    (void *)b->d_strip, (void *)b->d_out})
        (void)hipFree(p);
    delete b;
}

// Line length D of a system whose rows form lines (a grid numbered line by
// line): D is the largest column offset |col - row|, and applies when every
// offset is below D/4 or within D/4 of D and D >= kStripMinLine; else 0
// (phase A in row order).  Shorter lines keep their neighbour lines in the
// L2 in row order already.
constexpr int32_t kStripMinLine = 128;

int32_t strip_line(int32_t n, const int32_t *rp, const int32_t *ci) {
    int64_t D = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) D = std::max<int64_t>(D, std::llabs((int64_t)ci[k] - i));
    if (D < kStripMinLine || D > INT32_MAX / 4) return 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t o = std::llabs((int64_t)ci[k] - i);
            if (!(4 * o < D || 4 * o > 3 * D)) return 0;
        }
    return (int32_t)D;
}

int validate_sched(const cg_batch_sched *s) {
    if (!s) return fail(CG_EINVAL, "schedule is NULL");
    if (s->blocks_per_cu < 1 || s->blocks_per_cu > 64) return fail(CG_EINVAL, "blocks_per_cu must be in [1, 64]");
    if (s->rows_per_thread != 1 && s->rows_per_thread != 2) return fail(CG_EINVAL, "rows_per_thread must be 1 or 2");
    if (!(s->team_exponent >= 0.0 && s->team_exponent <= 3.0))
        return fail(CG_EINVAL, "team_exponent must be in [0, 3]");
    if (s->max_team < 0) return fail(CG_EINVAL, "max_team must be >= 0");
    if (s->rhs_per_lane < 0 || s->rhs_per_lane > 2) return fail(CG_EINVAL, "rhs_per_lane must be 0, 1 or 2");
    if (s->launch != CG_BATCH_LAUNCH_COOPERATIVE && s->launch != CG_BATCH_LAUNCH_ORDINARY)
        return fail(CG_EINVAL, "launch must be CG_BATCH_LAUNCH_COOPERATIVE or CG_BATCH_LAUNCH_ORDINARY");
    return CG_OK;
}

int lanes_variant(const cg_batch *b, const cg_batch_sched &s) {
    return (s.rhs_per_lane == 1 || (b->nrhs & 1)) ? 1 : 2;
}

// Workgroups per system, with w_k = n_k^exponent as a system's cost: the
// smallest per-workgroup load L for which the batch fits the grid, where a
// system heavier than L gets ceil(w_k / L) workgroups of its own (at most one
// per 16 rows, at most max_team) and the lighter ones share workgroups of
// capacity L (first fit, heaviest first; a workgroup then solves its systems
// one after another).  Workgroups left over go, one at a time, to the team
// with the largest load per workgroup that may still grow.  With few systems
// every one is heavier than L and has a team of its own.
int assign_teams(cg_batch *b, const cg_batch_sched &s) {
    const int occ = batch_blocks_per_cu(s.rows_per_thread, lanes_variant(b, s));
    if (occ <= 0) return fail(CG_EDEVICE, "occupancy query of the batched kernel failed");
    int grid = std::min(s.blocks_per_cu, occ) * b->cus;
    grid = std::max(1, std::min(grid, b->grid_cap));
    const int nsys = b->nsys;
    std::vector<double> wgt(nsys);
    std::vector<int32_t> cap(nsys);
    double wsum = 0.0, wmax = 0.0;
    for (int k = 0; k < nsys; ++k) {
        const int64_t n = b->row_off[k + 1] - b->row_off[k];
        wgt[k] = std::pow((double)std::max<int64_t>(n, 1), s.team_exponent);
        wsum += wgt[k];
        wmax = std::max(wmax, wgt[k]);
        int64_t c = std::max<int64_t>(1, n / kBatchRowsPerStep);
        if (s.max_team > 0) c = std::min<int64_t>(c, s.max_team);
        cap[k] = (int32_t)std::min<int64_t>(c, grid);
    }
    std::vector<int> order(nsys);
    for (int k = 0; k < nsys; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return wgt[x] > wgt[y]; });
    std::vector<int32_t> T(nsys), bin_of(nsys);
    // First fit over the shared workgroups: a tree of the smallest load in
    // each range of bins finds the leftmost bin with load + w <= L in
    // O(log grid) (a rounded sum is monotone in the load, so the subtree
    // test is exact); bins not yet opened hold load 0.
    int leaves = 1;
    while (leaves < grid + 1) leaves <<= 1;
    std::vector<double> tree(2 * (size_t)leaves);
    int nbins = 0;
    // workgroups used at load L (T, bin_of, tree and nbins filled in);
    // stops early, returning grid + 1, once the plan cannot fit the grid
    auto plan = [&](double L) -> int64_t {
        int64_t used = 0;
        std::fill(tree.begin(), tree.end(), 0.0);
        nbins = 0;
        for (int k : order) {
            if (wgt[k] > L) {   // heavier than L: a team of its own (these come first)
                T[k] = (int32_t)std::min<int64_t>(cap[k], (int64_t)std::ceil(wgt[k] / L));
                bin_of[k] = -1;
                used += T[k];
                if (used > grid) return (int64_t)grid + 1;
                continue;
            }
            T[k] = 1;
            size_t v = 1;
            while (v < (size_t)leaves) v = tree[2 * v] + wgt[k] <= L ? 2 * v : 2 * v + 1;
            const int i = (int)(v - (size_t)leaves);
            if (i >= nbins) nbins = i + 1;
            if (used + nbins > grid) return (int64_t)grid + 1;
            tree[v] += wgt[k];
            for (v >>= 1; v >= 1; v >>= 1) tree[v] = std::min(tree[2 * v], tree[2 * v + 1]);
            bin_of[k] = i;
        }
        return used + nbins;
    };
    // smallest load limit that fits: any L >= wmax places every system in
    // shared workgroups, and L = wsum needs only one
    double lo = wsum / grid, hi = std::max(wmax, lo);
    if (plan(hi) > grid) hi = std::max(hi, 2.0 * wsum);
    if (plan(lo) > grid)
        for (int it = 0; it < 60; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (plan(mid) <= grid) hi = mid;
            else lo = mid;
        }
    else
        hi = lo;
    int64_t used = plan(hi);
    if (used > grid) return fail(CG_EDEVICE, "team assignment exceeds the grid");
    while (used < grid) {
        int best = -1;
        for (int k : order)
            if (bin_of[k] < 0 && T[k] < cap[k] && (best < 0 || wgt[k] / T[k] > wgt[best] / T[best])) best = k;
        if (best < 0) break;
        ++T[best];
        ++used;
    }
    // workgroups: the teams of their own (in system order), then the shared ones
    std::vector<int32_t> wg_item((size_t)used + 1), item_sys, item_rank, first(nsys);
    std::vector<std::vector<int32_t>> in_bin((size_t)nbins);
    for (int k = 0; k < nsys; ++k)
        if (bin_of[k] >= 0) in_bin[(size_t)bin_of[k]].push_back(k);
    int w = 0;
    for (int k = 0; k < nsys; ++k) {
        if (bin_of[k] >= 0) continue;
        first[k] = w;
        for (int r = 0; r < T[k]; ++r, ++w) {
            wg_item[(size_t)w] = (int32_t)item_sys.size();
            item_sys.push_back(k);
            item_rank.push_back(r);
        }
    }
    for (int i = 0; i < nbins; ++i, ++w) {
        wg_item[(size_t)w] = (int32_t)item_sys.size();
        for (int k : in_bin[(size_t)i]) {
            first[k] = w;
            item_sys.push_back(k);
            item_rank.push_back(0);
        }
    }
    wg_item[(size_t)used] = (int32_t)item_sys.size();
    if (w != used || (int64_t)item_sys.size() > b->item_cap)
        return fail(CG_EDEVICE, "team assignment exceeds the grid");
    HIP_TRY(hipMemcpy(b->d_wg_item, wg_item.data(), sizeof(int32_t) * ((size_t)used + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_item_sys, item_sys.data(), sizeof(int32_t) * item_sys.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_item_rank, item_rank.data(), sizeof(int32_t) * item_rank.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_team_first, first.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_team_size, T.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice));
    b->grid = (int)used;
    b->team_size = T;
    b->sched = s;
    return CG_OK;
}

}  // namespace

extern "C" void cg_batch_default_sched(cg_batch_sched *s) {
    if (!s) return;
    s->blocks_per_cu = 4;
    s->rows_per_thread = 1;
    s->team_exponent = 1.0;
    s->max_team = 0;
    s->rhs_per_lane = 0;
    s->launch = CG_BATCH_LAUNCH_COOPERATIVE;
}

extern "C" int cg_batch_create(int32_t nsys, const int32_t *n, const int64_t *nnz,
                               const int32_t *const *row_ptr, const int32_t *const *col,
                               const double *const *val, int32_t nrhs, cg_batch **out) {
    clear_error();
    if (!out) return fail(CG_EINVAL, "out is NULL");
    *out = nullptr;
    if (nsys <= 0) return fail(CG_EINVAL, "nsys must be >= 1");
    if (nrhs < 1 || nrhs > CG_BATCH_MAX_RHS) return fail(CG_EINVAL, "nrhs must be in [1, %d]", CG_BATCH_MAX_RHS);
    if (!n || !nnz || !row_ptr || !col || !val) return fail(CG_EINVAL, "NULL argument");
    int64_t rows = 0, ents = 0;
    for (int32_t k = 0; k < nsys; ++k) {
        if (n[k] <= 0) return fail(CG_EINVAL, "system %d is empty", k);
        const int rc = validate_csr(n[k], nnz[k], row_ptr[k], col[k], val[k]);
        if (rc) return rc;
        rows += n[k];
        ents += nnz[k];
    }
    if (rows >= INT32_MAX || ents >= INT32_MAX) return fail(CG_EINVAL, "stacked systems exceed int32 indices");
    if (rows * (int64_t)nrhs >= ((int64_t)1 << 40)) return fail(CG_EINVAL, "vectors too large");
    cg_batch *b = new (std::nothrow) cg_batch();
    if (!b) return fail(CG_ENOMEM, "out of host memory");
    auto bail = [&](int code) {
        batch_free(b);
        return code;
    };
    if (hipGetDevice(&b->dev) != hipSuccess) return bail(fail(CG_EDEVICE, "no HIP device"));
    b->cus = device_cu_count();
    b->nsys = nsys;
    b->nrhs = nrhs;
    b->n_total = rows;
    b->nnz_total = ents;
    std::vector<int32_t> rp, ci;
    std::vector<double> va;
    try {
        b->row_off.assign((size_t)nsys + 1, 0);
        rp.resize((size_t)rows + 1);
        ci.resize((size_t)ents);
        va.resize((size_t)ents);
    } catch (...) {
        return bail(fail(CG_ENOMEM, "out of host memory"));
    }
    int64_t r = 0, z = 0;
    for (int32_t k = 0; k < nsys; ++k) {
        b->row_off[k] = r;
        for (int32_t i = 0; i < n[k]; ++i) rp[r + i] = (int32_t)(z + row_ptr[k][i]);
        for (int64_t e = 0; e < nnz[k]; ++e) {
            ci[z + e] = (int32_t)(r + col[k][e]);
            va[z + e] = val[k][e];
        }
        r += n[k];
        z += nnz[k];
    }
    b->row_off[nsys] = r;
    rp[r] = (int32_t)z;
    int occ = 0;
    for (int u = 1; u <= 2; ++u)
        for (int v = 1; v <= 2; ++v) occ = std::max(occ, batch_blocks_per_cu(u, v));
    if (occ <= 0) return bail(fail(CG_EDEVICE, "occupancy query of the batched kernel failed"));
    b->grid_cap = occ * b->cus;
    const size_t vec = (size_t)rows * nrhs;
    hipError_t e = dmalloc(&b->d_rp, (size_t)rows + 1);
    if (e == hipSuccess) e = dmalloc(&b->d_ci, (size_t)ents);
    if (e == hipSuccess) e = dmalloc(&b->d_val, (size_t)ents);
    if (e == hipSuccess) e = dmalloc(&b->d_R, vec);
    if (e == hipSuccess) e = dmalloc(&b->d_P, vec);
    if (e == hipSuccess) e = dmalloc(&b->d_Q, vec);
    if (e == hipSuccess) e = dmalloc(&b->d_part, (size_t)b->grid_cap * kBatchSlots * kBatchLanes);
    if (e == hipSuccess) e = dmalloc(&b->d_bar, (size_t)nsys);
    if (e == hipSuccess) e = dmalloc(&b->d_err, 1);
    if (e == hipSuccess) e = dmalloc(&b->d_episodes, (size_t)nsys);
    b->item_cap = (int64_t)b->grid_cap + nsys;   // one item per team member plus one per shared system
    if (e == hipSuccess) e = dmalloc(&b->d_wg_item, (size_t)b->grid_cap + 1);
    if (e == hipSuccess) e = dmalloc(&b->d_item_sys, (size_t)b->item_cap);
    if (e == hipSuccess) e = dmalloc(&b->d_item_rank, (size_t)b->item_cap);
    if (e == hipSuccess) e = dmalloc(&b->d_team_first, (size_t)nsys);
    if (e == hipSuccess) e = dmalloc(&b->d_team_size, (size_t)nsys);
    if (e == hipSuccess) e = dmalloc(&b->d_row_off, (size_t)nsys + 1);
    if (e == hipSuccess) e = dmalloc(&b->d_strip, (size_t)nsys);
    if (e == hipSuccess) e = dmalloc(&b->d_out, (size_t)nsys * nrhs);
    if (e != hipSuccess) return bail(fail(CG_ENOMEM, "batch allocation failed: %s", hipGetErrorString(e)));
    e = hipMemcpy(b->d_rp, rp.data(), sizeof(int32_t) * rp.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && ents) e = hipMemcpy(b->d_ci, ci.data(), sizeof(int32_t) * ci.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && ents) e = hipMemcpy(b->d_val, va.data(), sizeof(double) * va.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_row_off, b->row_off.data(), sizeof(int64_t) * b->row_off.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        std::vector<int32_t> strip((size_t)nsys);
#pragma omp parallel for schedule(dynamic)
        for (int32_t k = 0; k < nsys; ++k) strip[(size_t)k] = strip_line(n[k], row_ptr[k], col[k]);
        e = hipMemcpy(b->d_strip, strip.data(), sizeof(int32_t) * strip.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return bail(fail(CG_EDEVICE, "batch upload failed: %s", hipGetErrorString(e)));
    cg_batch_sched s;
    cg_batch_default_sched(&s);
    const int rc = assign_teams(b, s);
    if (rc) return bail(rc);
    *out = b;
    return CG_OK;
}

extern "C" void cg_batch_destroy(cg_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->dev);
    (void)(b->stream ? hipStreamSynchronize(b->stream) : hipDeviceSynchronize());
    batch_free(b);
}

extern "C" int cg_batch_set_stream(cg_batch *b, void *hip_stream) {
    clear_error();
    if (!b) return fail(CG_EINVAL, "batch is NULL");
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return CG_OK;
}

extern "C" int cg_batch_layout(const cg_batch *b, int64_t *row_offset) {
    clear_error();
    if (!b || !row_offset) return fail(CG_EINVAL, "NULL argument");
    std::memcpy(row_offset, b->row_off.data(), sizeof(int64_t) * b->row_off.size());
    return CG_OK;
}

extern "C" int cg_batch_set_sched(cg_batch *b, const cg_batch_sched *s) {
    clear_error();
    if (!b) return fail(CG_EINVAL, "batch is NULL");
    int rc = validate_sched(s);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(b->dev));
    HIP_TRY(b->stream ? hipStreamSynchronize(b->stream) : hipDeviceSynchronize());
    return assign_teams(b, *s);
}

extern "C" int cg_batch_get_sched(const cg_batch *b, cg_batch_sched *s) {
    clear_error();
    if (!b || !s) return fail(CG_EINVAL, "NULL argument");
    *s = b->sched;
    return CG_OK;
}

extern "C" int cg_batch_solve(cg_batch *b, const double *B, double *X, double tol, int32_t maxit,
                              cg_batch_result *res, cg_batch_stats *stats) {
    clear_error();
    if (!b) return fail(CG_EINVAL, "batch is NULL");
    if (!B || !X) return fail(CG_EINVAL, "B/X is NULL");
    if (!(tol >= 0.0)) return fail(CG_EINVAL, "tol must be >= 0");
    if (maxit < 0) return fail(CG_EINVAL, "maxit must be >= 0");
    HIP_TRY(hipSetDevice(b->dev));
    hipStream_t st = b->stream;
    HIP_TRY(hipMemsetAsync(b->d_bar, 0, sizeof(int32_t) * b->nsys, st));
    HIP_TRY(hipMemsetAsync(b->d_err, 0, sizeof(int32_t), st));
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, b->dev) != hipSuccess || rate_khz <= 0)
        rate_khz = 100000;
    BatchArgs a{};
    a.rp = b->d_rp;
    a.ci = b->d_ci;
    a.val = b->d_val;
    a.B = B;
    a.X = X;
    a.R = b->d_R;
    a.P = b->d_P;
    a.Q = b->d_Q;
    a.part = b->d_part;
    a.bar = b->d_bar;
    a.err = b->d_err;
    a.wg_item = b->d_wg_item;
    a.item_sys = b->d_item_sys;
    a.item_rank = b->d_item_rank;
    a.team_first = b->d_team_first;
    a.team_size = b->d_team_size;
    a.row_off = b->d_row_off;
    a.strip = b->d_strip;
    a.out = b->d_out;
    a.episodes = b->d_episodes;
    a.nrhs = b->nrhs;
    a.maxit = maxit;
    a.tol = tol;
    a.timeout_ticks = (int64_t)rate_khz * 1000 * 20;   // 20 s for one team wait
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
    int V = lanes_variant(b, b->sched);
    if (V == 2 && ((reinterpret_cast<uintptr_t>(B) | reinterpret_cast<uintptr_t>(X)) & 15)) {
        // unaligned vectors: one right-hand side per lane, if that variant
        // keeps the grid resident
        if (batch_blocks_per_cu(b->sched.rows_per_thread, 1) * b->cus < b->grid) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return fail(CG_EINVAL, "B and X must be 16-byte aligned for this schedule");
        }
        V = 1;
    }
    // the grid is within the kernel's occupancy (assign_teams), so every
    // workgroup is resident at once in either launch form
    const hipError_t le = launch_batch_cg(a, b->grid, b->sched.rows_per_thread, V,
                                          b->sched.launch == CG_BATCH_LAUNCH_COOPERATIVE, st);
    if (le != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return fail(CG_EDEVICE, "persistent launch of %d workgroups failed: %s", b->grid, hipGetErrorString(le));
    }
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int32_t err = 0;
    HIP_TRY(hipMemcpy(&err, b->d_err, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (err) return fail(CG_EDEVICE, "a team barrier timed out; the launch was abandoned");
    std::vector<BatchOutDev> o((size_t)b->nsys * b->nrhs);
    std::vector<int32_t> ep(b->nsys);
    HIP_TRY(hipMemcpy(o.data(), b->d_out, sizeof(BatchOutDev) * o.size(), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ep.data(), b->d_episodes, sizeof(int32_t) * ep.size(), hipMemcpyDeviceToHost));
    int rc = CG_OK;
    for (const BatchOutDev &r : o) {
        if (r.status == CG_EBREAKDOWN) rc = CG_EBREAKDOWN;
        else if (r.status == CG_MAXIT && rc == CG_OK) rc = CG_MAXIT;
    }
    if (res)
        for (size_t i = 0; i < o.size(); ++i) {
            res[i].status = o[i].status;
            res[i].iterations = o[i].iterations;
            res[i].rel_res_recur = o[i].rel_res_recur;
            res[i].rel_res_true = o[i].rel_res_true;
        }
    if (stats) {
        stats->t_kernel = 1e-3 * ms;
        stats->grid = b->grid;
        int multi = 0, mx = 0, bar = 0;
        for (int k = 0; k < b->nsys; ++k) {
            multi += b->team_size[k] > 1;
            if (b->team_size[k] > mx) {
                mx = b->team_size[k];
                bar = ep[k];
            }
        }
        stats->teams_multi = multi;
        stats->max_team = mx;
        stats->barriers = bar;
    }
    if (rc == CG_EBREAKDOWN) fail(CG_EBREAKDOWN, "some right-hand side broke down (p^T q <= 0 or not finite)");
    return rc;
}
