// cgmi.cpp -- host runtime of libcgmi: C ABI, CSR validation, row split, the
// GPU-only solve loops (float64 and mixed precision) and the split
// (coscheduled) solve with the host complement on OpenMP threads.  The device
// matrix and its SpMV schedule are in devmatrix.cpp, the preconditioned solve
// in fsai.cpp, the batched solve in batch.cpp.
//
// Section 3.2: the GPU owns the contiguous row block [row_begin, row_end);
// the host owns the rest.  Section 3.3: one host thread drives the GPU while
// host threads compute the host rows; barriers and device synchronisations
// are kept where a reduction or the visibility of p needs them.
// Section 3.4 (explicit copy): the GPU-owned segment of p is copied to the
// host and the host-owned segments to the device after every p update.
#include <hip/hip_runtime_api.h>
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/cgmi.h"
#include "cgmi_host.h"
#include "util_internal.h"
#include "cgmi_internal.h"

using namespace cgmi;

namespace {
thread_local std::string g_err;
}  // namespace

namespace cgmi {

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }
const char *error_message() { return g_err.c_str(); }

double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace cgmi

#define HIP_TRY(expr) CGMI_HIP_TRY(expr)

// ---------------------------------------------------------------------------
// validation and schedule

int cgmi::validate_csr(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                       const double *val) {
    if (n < 0) return fail(CG_EINVAL, "n must be >= 0 (got %d)", n);
    if (nnz < 0 || nnz > INT32_MAX) return fail(CG_EINVAL, "nnz out of int32 range");
    if (n > 0 && !rp) return fail(CG_EINVAL, "row_ptr is NULL");
    if (nnz > 0 && (!ci || !val)) return fail(CG_EINVAL, "col_idx/val is NULL");
    if (n == 0) return nnz == 0 ? CG_OK : fail(CG_EINVAL, "n = 0 but nnz != 0");
    if (rp[0] != 0) return fail(CG_EINVAL, "row_ptr[0] must be 0");
    if ((int64_t)rp[n] != nnz) return fail(CG_EINVAL, "row_ptr[n] = %d != nnz", rp[n]);
    for (int32_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return fail(CG_EINVAL, "row_ptr decreases at row %d", i);
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] < 0 || ci[k] >= n)
                return fail(CG_EINVAL, "column %d out of range in row %d", ci[k], i);
            if (k > rp[i] && ci[k] <= ci[k - 1])
                return fail(CG_EINVAL, "columns not strictly increasing in row %d", i);
        }
    }
    return CG_OK;
}

// SpMV schedule of the GPU block for the current options.
static int apply_schedule(cg_handle *h) {
    return dm_schedule(h->A, h->opts.spmv_kind, h->opts.spmv_grid, h->cus, h->grid_cap,
                       h->opts.precision == CG_PREC_MIXED, h->opts.spmv_colblock);
}

// The spmv_kind code of the tiling in use (cg_result.spmv_kind).
static int kind_code(const DevMatrix &A) {
    static const int code[6] = {1, 2, 3, 4, 5, 6};   // kTileVector .. kTileStencil
    return A.sched.kind == kTileSliced && A.use_gap ? 7 : code[A.sched.kind];
}

// float32 inner vectors of mixed precision (the float32 matrix copies are
// made by dm_schedule).
static int ensure_mixed_vectors(cg_handle *h) {
    if (h->d_r32) return CG_OK;
    hipError_t e = dmalloc(&h->d_r32, (size_t)h->m + 2);
    if (e == hipSuccess) e = dmalloc(&h->d_p32, (size_t)h->n + 2);
    if (e == hipSuccess) e = dmalloc(&h->d_q32, (size_t)h->m + 2);
    if (e != hipSuccess) return fail(CG_ENOMEM, "mixed-precision vectors: %s", hipGetErrorString(e));
    return CG_OK;
}

static void free_shared_p(cg_handle *h) {
    if (h->shared_mode == CG_EXCHANGE_MAPPED && h->h_pshared) hipHostFree(h->h_pshared);
    if (h->shared_mode == CG_EXCHANGE_MANAGED && h->d_pshared) hipFree(h->d_pshared);
    h->h_pshared = h->d_pshared = nullptr;
    h->shared_mode = -1;
}

// Allocate p where the host and the GPU both address it (Section 3.4 mapped
// and managed modes): page-locked coherent host memory mapped into the
// device's address space, or managed memory.  Zero-filled by the host.
static int ensure_shared_p(cg_handle *h, int mode) {
    if (h->shared_mode == mode) return CG_OK;
    free_shared_p(h);
    const size_t bytes = sizeof(double) * ((size_t)h->n + 2);
    if (mode == CG_EXCHANGE_MAPPED) {
        void *hp = nullptr, *dp = nullptr;
        if (hipHostMalloc(&hp, bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
            return fail(CG_ENOMEM, "mapped host allocation of p failed");
        if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess) {
            hipHostFree(hp);
            return fail(CG_EDEVICE, "no device address for the mapped p");
        }
        h->h_pshared = static_cast<double *>(hp);
        h->d_pshared = static_cast<double *>(dp);
    } else {
        int managed = 0;
        HIP_TRY(hipDeviceGetAttribute(&managed, hipDeviceAttributeManagedMemory, h->dev));
        if (!managed) return fail(CG_EINVAL, "the device reports no managed-memory support");
        void *mp = nullptr;
        const size_t granule = 4096;   // managed allocations come in 4 KiB pages
        if (hipMallocManaged(&mp, (bytes + granule - 1) / granule * granule, hipMemAttachGlobal) != hipSuccess)
            return fail(CG_ENOMEM, "managed allocation of p failed");
        h->h_pshared = h->d_pshared = static_cast<double *>(mp);
    }
    h->shared_mode = mode;
    std::memset(h->h_pshared, 0, bytes);
    return CG_OK;
}

static void free_device(cg_handle *h) {
    free_shared_p(h);
    fsai_free(h);
    dm_free(h->A);
    dm_free(h->G);
    dm_free(h->GT);
    hipFree(h->d_t); hipFree(h->d_z); hipFree(h->d_r2);
    hipFree(h->d_r32); hipFree(h->d_p32); hipFree(h->d_q32);
    hipFree(h->d_pbuf); hipFree(h->d_p2); hipFree(h->d_x); hipFree(h->d_r); hipFree(h->d_q);
    hipFree(h->d_vin); hipFree(h->d_vout);
    hipFree(h->d_part_setup); hipFree(h->d_part_pq); hipFree(h->d_part_rr); hipFree(h->d_part_rz);
    hipFree(h->d_state);
    hipFree(h->d_halo_d2h); hipFree(h->d_halo_h2d); hipFree(h->d_pack_d2h); hipFree(h->d_pack_h2d);
    if (h->h_state) hipHostFree(h->h_state);
    if (h->h_p) hipHostFree(h->h_p);
    if (h->h_pack_d2h) hipHostFree(h->h_pack_d2h);
    if (h->h_pack_h2d) hipHostFree(h->h_pack_h2d);
    if (h->s_d2h) hipStreamDestroy(h->s_d2h);
    if (h->s_h2d) hipStreamDestroy(h->s_h2d);
}

extern "C" void cg_default_opts(cg_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->precision = CG_PREC_FP64;
    o->precond = CG_PC_NONE;
    o->exchange = CG_EXCHANGE_WHOLE;
    o->host_threads = 0;
    o->check_every = 32;
    o->profile = 0;
    o->small_path = 1;
    o->spmv_grid = 0;
    o->spmv_kind = 0;
    o->spmv_colblock = 0;
    o->refine_delta = 0.01;
    o->vectors = CG_VECTORS_DEVICE;
    o->fuse_dir = CG_FUSE_AUTO;
}

extern "C" const char *cg_last_error(void) { return error_message(); }

extern "C" int cg_create(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                         const double *val, int32_t row_begin, int32_t row_end, cg_handle **out) {
    clear_error();
    if (!out) return fail(CG_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_csr(n, nnz, row_ptr, col_idx, val);
    if (rc) return rc;
    if (row_begin < 0 || row_end < row_begin || row_end > n)
        return fail(CG_EINVAL, "row range [%d, %d) not inside [0, %d)", row_begin, row_end, n);
    cg_handle *h = new (std::nothrow) cg_handle();
    if (!h) return fail(CG_ENOMEM, "out of host memory");
    cg_default_opts(&h->opts);
    h->n = n;
    h->nnz = nnz;
    h->rb = row_begin;
    h->re = row_end;
    h->m = row_end - row_begin;
    try {
        h->h_rp.resize((size_t)n + 1);
        par_copy(h->h_rp.data(), row_ptr, (size_t)n + 1);
        h->h_ci.resize((size_t)nnz);
        par_copy(h->h_ci.data(), col_idx, (size_t)nnz);
        h->h_val.resize((size_t)nnz);
        par_copy(h->h_val.data(), val, (size_t)nnz);
    } catch (...) {
        delete h;
        return fail(CG_ENOMEM, "out of host memory copying the matrix");
    }
    h->nnz_gpu = (int64_t)h->h_rp[h->re] - h->h_rp[h->rb];
    h->nnz_cpu = nnz - h->nnz_gpu;
    auto bail = [&](int code) {
        free_device(h);
        delete h;
        return code;
    };
    {
        // A host-only handle (row_begin == row_end: the paper's CPU-only
        // configuration) needs no device; without one it runs on host
        // threads alone and takes host vectors.  Any GPU rows need a device.
        int count = 0;
        const bool have_dev = hipGetDeviceCount(&count) == hipSuccess && count > 0 &&
                              hipGetDevice(&h->dev) == hipSuccess;
        if (!have_dev && h->m == 0 && n > 0) {
            h->nodev = true;
            h->dev = -1;
            h->opts.vectors = CG_VECTORS_HOST;
            try {
                h->h_x.assign(n, 0.0);
                h->h_r.assign(n, 0.0);
                h->h_q.assign(n, 0.0);
                h->h_b.assign(n, 0.0);
                h->h_p_store.assign(n, 0.0);
            } catch (...) {
                delete h;
                return fail(CG_ENOMEM, "out of host memory");
            }
            h->h_p = h->h_p_store.data();
            *out = h;
            return CG_OK;
        }
        if (!have_dev) {
            delete h;
            return fail(CG_EDEVICE, "no HIP device (rows [%d, %d) are to run on the GPU)", row_begin, row_end);
        }
    }
    // device address of the static scratch of cg_solve_noalloc, once per
    // device (a failure is kept and reported by that entry point)
    (void)scratch_setup();
    h->cus = device_cu_count();
    const int m = h->m;
    // device copy of the GPU row block, row pointers rebased (Section 3.2)
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    {
        const int rc2 = dm_upload(h->A, m, h->h_rp.data() + h->rb, h->h_ci.data(), h->h_val.data(), h->rb);
        if (rc2) return bail(rc2);
    }
    chk(dmalloc(&h->d_pbuf, (size_t)n + 2));
    chk(dmalloc(&h->d_x, (size_t)m + 1));
    chk(dmalloc(&h->d_r, (size_t)m + 1));
    chk(dmalloc(&h->d_q, (size_t)m + 1));
    // vector kernels: pairs of rows per thread, at most 4 workgroups per CU
    // (fewer partials for the next kernel to sum; measured as fast as 8 per CU
    // at 256^3 and 9% faster per PCG iteration at 1024^2)
    h->vec_grid = std::max(1, std::min(h->cus * 4, (int)(((int64_t)m / 2 + kBlock - 1) / kBlock)));
    h->grid_cap = std::max(h->cus * 16, 64);
    chk(dmalloc(&h->d_part_setup, 2 * (size_t)h->grid_cap));
    chk(dmalloc(&h->d_part_pq, (size_t)h->grid_cap));
    chk(dmalloc(&h->d_part_rr, (size_t)h->grid_cap));
    chk(dmalloc(&h->d_part_rz, (size_t)h->grid_cap));
    try { h->h_part.assign(2 * (size_t)h->grid_cap, 0.0); } catch (...) { return bail(fail(CG_ENOMEM, "out of host memory")); }
    chk(dmalloc(&h->d_state, 1));
    if (e != hipSuccess) return bail(fail(CG_ENOMEM, "device allocation failed: %s", hipGetErrorString(e)));
    if (hipHostMalloc(reinterpret_cast<void **>(&h->h_state), sizeof(DevState)) != hipSuccess)
        return bail(fail(CG_ENOMEM, "pinned allocation failed"));
    // p + rb must be 16-byte aligned for the paired loads of the update kernels
    h->d_p = h->d_pbuf + (h->rb & 1);
    {
        const int rc2 = apply_schedule(h);
        if (rc2) return bail(rc2);
    }
    chk(hipMemset(h->d_state, 0, sizeof(DevState)));
    chk(hipMemset(h->d_pbuf, 0, sizeof(double) * ((size_t)n + 2)));
    if (e != hipSuccess) return bail(fail(CG_EDEVICE, "upload failed: %s", hipGetErrorString(e)));
    if (!h->gpu_only() && n > 0) {
        // split or host-only: host vectors, pinned p, exchange streams, halo lists
        try {
            h->h_x.assign(n, 0.0);
            h->h_r.assign(n, 0.0);
            h->h_q.assign(n, 0.0);
            h->h_b.assign(n, 0.0);
        } catch (...) {
            return bail(fail(CG_ENOMEM, "out of host memory"));
        }
        if (hipHostMalloc(reinterpret_cast<void **>(&h->h_p), sizeof(double) * (size_t)n) != hipSuccess)
            return bail(fail(CG_ENOMEM, "pinned allocation failed"));
        std::memset(h->h_p, 0, sizeof(double) * (size_t)n);
        if (m > 0) {
            chk(hipStreamCreateWithFlags(&h->s_d2h, hipStreamNonBlocking));
            chk(hipStreamCreateWithFlags(&h->s_h2d, hipStreamNonBlocking));
            // halo: host-owned columns read by GPU rows, GPU-owned columns read by host rows
            std::vector<char> mark((size_t)n, 0);
            for (int64_t k = h->h_rp[h->rb]; k < h->h_rp[h->re]; ++k) {
                const int32_t c = h->h_ci[k];
                if (c < h->rb || c >= h->re) mark[c] = 1;
            }
            for (int32_t c = 0; c < n; ++c) if (mark[c]) h->halo_h2d.push_back(c);
            std::fill(mark.begin(), mark.end(), 0);
            for (int32_t i = 0; i < n; ++i) {
                if (i >= h->rb && i < h->re) continue;
                for (int32_t k = h->h_rp[i]; k < h->h_rp[i + 1]; ++k) {
                    const int32_t c = h->h_ci[k];
                    if (c >= h->rb && c < h->re) mark[c] = 1;
                }
            }
            for (int32_t c = 0; c < n; ++c) if (mark[c]) h->halo_d2h.push_back(c);
            const size_t a = h->halo_d2h.size(), b = h->halo_h2d.size();
            chk(dmalloc(&h->d_halo_d2h, a));
            chk(dmalloc(&h->d_halo_h2d, b));
            chk(dmalloc(&h->d_pack_d2h, a));
            chk(dmalloc(&h->d_pack_h2d, b));
            if (e == hipSuccess && a)
                chk(hipMemcpy(h->d_halo_d2h, h->halo_d2h.data(), sizeof(int32_t) * a, hipMemcpyHostToDevice));
            if (e == hipSuccess && b)
                chk(hipMemcpy(h->d_halo_h2d, h->halo_h2d.data(), sizeof(int32_t) * b, hipMemcpyHostToDevice));
            if (e == hipSuccess)
                chk(hipHostMalloc(reinterpret_cast<void **>(&h->h_pack_d2h), sizeof(double) * (a ? a : 1)));
            if (e == hipSuccess)
                chk(hipHostMalloc(reinterpret_cast<void **>(&h->h_pack_h2d), sizeof(double) * (b ? b : 1)));
            if (e != hipSuccess) return bail(fail(CG_EDEVICE, "split-mode setup failed: %s", hipGetErrorString(e)));
        }
    }
    *out = h;
    return CG_OK;
}

extern "C" void cg_destroy(cg_handle *h) {
    if (!h) return;
    if (h->nodev) {
        delete h;
        return;
    }
    hipSetDevice(h->dev);
    if (h->stream) hipStreamSynchronize(h->stream);
    else hipDeviceSynchronize();
    free_device(h);
    delete h;
}

extern "C" int cg_set_stream(cg_handle *h, void *hip_stream) {
    if (!h) return fail(CG_EINVAL, "handle is NULL");
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return CG_OK;
}

extern "C" int cg_set_opts(cg_handle *h, const cg_opts *o) {
    if (!h || !o) return fail(CG_EINVAL, "NULL argument");
    if (o->precision != CG_PREC_FP64 && o->precision != CG_PREC_MIXED)
        return fail(CG_EINVAL, "unknown precision %d", o->precision);
    if (o->precond != CG_PC_NONE && o->precond != CG_PC_FSAI)
        return fail(CG_EINVAL, "unknown preconditioner %d", o->precond);
    if (o->exchange < CG_EXCHANGE_WHOLE || o->exchange > CG_EXCHANGE_MANAGED)
        return fail(CG_EINVAL, "unknown exchange mode %d", o->exchange);
    const bool shared = o->exchange == CG_EXCHANGE_MAPPED || o->exchange == CG_EXCHANGE_MANAGED;
    if (shared && (o->precision != CG_PREC_FP64 || o->precond != CG_PC_NONE))
        return fail(CG_EINVAL, "mapped and managed p need float64 CG without preconditioner");
    if (o->check_every < 1) return fail(CG_EINVAL, "check_every must be >= 1");
    if (o->host_threads < 0) return fail(CG_EINVAL, "host_threads must be >= 0");
    if (o->spmv_grid < 0) return fail(CG_EINVAL, "spmv_grid must be >= 0");
    if (!(o->refine_delta > 0.0 && o->refine_delta < 1.0))
        return fail(CG_EINVAL, "refine_delta must be in (0, 1)");
    if ((o->precision != CG_PREC_FP64 || o->precond != CG_PC_NONE) && !h->gpu_only())
        return fail(CG_EINVAL, "mixed precision and preconditioning need a GPU-only handle");
    if (o->spmv_kind < 0 || o->spmv_kind > 7) return fail(CG_EINVAL, "unknown spmv_kind %d", o->spmv_kind);
    if (o->spmv_colblock < 0) return fail(CG_EINVAL, "spmv_colblock must be >= 0");
    if (o->vectors != CG_VECTORS_DEVICE && o->vectors != CG_VECTORS_HOST)
        return fail(CG_EINVAL, "vectors must be CG_VECTORS_DEVICE or CG_VECTORS_HOST");
    if (o->fuse_dir < CG_FUSE_AUTO || o->fuse_dir > CG_FUSE_OFF)
        return fail(CG_EINVAL, "fuse_dir must be CG_FUSE_AUTO, CG_FUSE_ON or CG_FUSE_OFF");
    if (h->nodev) {
        // a host-only handle without a device: host vectors, p in host memory
        if (o->vectors != CG_VECTORS_HOST || shared)
            return fail(CG_EINVAL, "a handle without a device takes host vectors and keeps p in host memory");
        h->opts = *o;
        return CG_OK;
    }
    if (o->precision == CG_PREC_MIXED && o->precond != CG_PC_NONE)
        return fail(CG_EINVAL, "the preconditioned solve runs in float64 only");
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(h->stream ? hipStreamSynchronize(h->stream) : hipDeviceSynchronize());
    if (shared && h->n > 0) {
        const int rc0 = ensure_shared_p(h, o->exchange);
        if (rc0) return rc0;
    }
    h->opts = *o;
    int rc = apply_schedule(h);
    if (rc) return rc;
    if (o->precision == CG_PREC_MIXED) {
        rc = ensure_mixed_vectors(h);
        if (rc) return rc;
    }
    return CG_OK;
}

extern "C" int cg_get_opts(const cg_handle *h, cg_opts *o) {
    if (!h || !o) return fail(CG_EINVAL, "NULL argument");
    *o = h->opts;
    return CG_OK;
}

extern "C" int cg_slice_info(const cg_handle *h, int32_t *rows_gpu, int64_t *nnz_gpu) {
    if (!h) return fail(CG_EINVAL, "handle is NULL");
    if (rows_gpu) *rows_gpu = h->m;
    if (nnz_gpu) *nnz_gpu = h->nnz_gpu;
    return CG_OK;
}

extern "C" int cg_read_slice(const cg_handle *h, int32_t *row_ptr, int32_t *col_idx, double *val) {
    if (!h) return fail(CG_EINVAL, "handle is NULL");
    if (h->m == 0) {   // no GPU rows: the rebased row pointers are {0}
        if (row_ptr) row_ptr[0] = 0;
        return CG_OK;
    }
    HIP_TRY(hipSetDevice(h->dev));
    if (row_ptr) HIP_TRY(hipMemcpy(row_ptr, h->A.d_rp, sizeof(int32_t) * ((size_t)h->m + 1), hipMemcpyDeviceToHost));
    if (h->nnz_gpu && col_idx)
        HIP_TRY(hipMemcpy(col_idx, h->A.d_ci, sizeof(int32_t) * h->nnz_gpu, hipMemcpyDeviceToHost));
    if (h->nnz_gpu && val)
        HIP_TRY(hipMemcpy(val, h->A.d_val, sizeof(double) * h->nnz_gpu, hipMemcpyDeviceToHost));
    return CG_OK;
}

// ---------------------------------------------------------------------------
// host complement (Section 3.3: host threads share the host rows equally)

namespace {

struct HostRows {
    int32_t rb, re, n;
    int32_t count() const { return n - (re - rb); }
    int32_t row(int32_t v) const { return v < rb ? v : v - rb + re; }
};

int host_threads(const cg_handle *h) {
    int t = h->opts.host_threads > 0 ? h->opts.host_threads : omp_get_max_threads();
    return std::max(1, t);
}

// Per-thread partial sums are combined in thread order (deterministic for a
// fixed thread count).
template <class F>
double host_reduce(const cg_handle *h, F &&body) {
    const HostRows hr{h->rb, h->re, h->n};
    const int T = host_threads(h);
    std::vector<double> part((size_t)T, 0.0);
    const int32_t cnt = hr.count();
#pragma omp parallel num_threads(T)
    {
        const int t = omp_get_thread_num();
        const int nt = omp_get_num_threads();
        const int32_t lo = (int32_t)((int64_t)cnt * t / nt), hi = (int32_t)((int64_t)cnt * (t + 1) / nt);
        double acc = 0.0;
        for (int32_t v = lo; v < hi; ++v) acc += body(hr.row(v));
        part[t] = acc;
    }
    double s = 0.0;
    for (int t = 0; t < T; ++t) s += part[t];
    return s;
}

double host_row_dot(const cg_handle *h, int32_t i, const double *p) {
    double s = 0.0;
    for (int32_t k = h->h_rp[i]; k < h->h_rp[i + 1]; ++k) s += h->h_val[k] * p[h->h_ci[k]];
    return s;
}

}  // namespace

// ---------------------------------------------------------------------------
// device helpers

namespace cgmi {

int gpu_state_init(cg_handle *h, double tol, int32_t maxit) {
    DevState &s = *h->h_state;
    std::memset(&s, 0, sizeof s);
    s.tol = tol;
    s.maxit = maxit;
    s.delta = h->opts.refine_delta;
    HIP_TRY(hipMemcpyAsync(h->d_state, h->h_state, sizeof(DevState), hipMemcpyHostToDevice, h->stream));
    return CG_OK;
}

int gpu_state_read(cg_handle *h) {
    HIP_TRY(hipMemcpyAsync(h->h_state, h->d_state, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CG_OK;
}

// Copy `count` partials (or two interleaved arrays of `count`) to the host and
// sum each in workgroup order.
int sum_partials_host(cg_handle *h, const double *d_part, int count, int arrays, double *s0,
                      double *s1) {
    HIP_TRY(hipMemcpyAsync(h->h_part.data(), d_part, sizeof(double) * (size_t)count * arrays,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    double a = 0.0, b = 0.0;
    for (int i = 0; i < count; ++i) a += h->h_part[i];
    if (arrays > 1)
        for (int i = 0; i < count; ++i) b += h->h_part[count + i];
    *s0 = a;
    if (s1) *s1 = b;
    return CG_OK;
}

// ||b - A x||^2 and ||b||^2 over the GPU rows (x full length on the device).
int gpu_true_residual(cg_handle *h, const double *b_own, const double *x_full, double *rr,
                      double *bb) {
    HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, h->A.grid, x_full, h->d_q, nullptr, b_own, h->d_q,
                        h->d_part_setup, no_partials(), no_partials(), nullptr, kSpmvResidual, 0,
                        h->stream));
    return sum_partials_host(h, h->d_part_setup, h->A.grid, 2, rr, bb);
}

int status_of(int done) {
    switch (done) {
        case kDoneConverged: return CG_OK;
        case kDoneBreakdown: return CG_EBREAKDOWN;
        default: return CG_MAXIT;
    }
}

}  // namespace cgmi

// ---------------------------------------------------------------------------
// GPU-only solve: alpha, beta and the stop test stay on the device; the host
// queues iterations in chunks and polls the device state between chunks.

namespace {

// Device buffers of one plain float64 GPU-only solve: the handle's own, or
// carved from the library's static scratch (cg_solve_noalloc).
struct PlainWork {
    double *x, *r, *q;        // n each: working x, residual, A p
    double *p, *p2;           // n each; p2 null: x updated every iteration from p
    double *part_setup;       // 2 x A.grid: r^T r, b^T b of the residual kernel
    double *part_pq;          // A.grid
    double *part_rr;          // vec_grid
    DevState *state;          // device state
    DevState *h_state;        // host copy, read at poll points
    bool events;              // HIP events allowed (SpMV timing, cg_opts.profile)
    bool state_kernel;        // initialise the state with a kernel (no host staging)
};

int work_state_init(cg_handle *h, const PlainWork &w, double tol, int32_t maxit) {
    if (w.state_kernel) {
        HIP_TRY(launch_state_init(w.state, tol, maxit, h->opts.refine_delta, h->stream));
        return CG_OK;
    }
    DevState &s = *w.h_state;
    std::memset(&s, 0, sizeof s);
    s.tol = tol;
    s.maxit = maxit;
    s.delta = h->opts.refine_delta;
    HIP_TRY(hipMemcpyAsync(w.state, w.h_state, sizeof(DevState), hipMemcpyHostToDevice, h->stream));
    return CG_OK;
}

int work_state_read(cg_handle *h, const PlainWork &w) {
    HIP_TRY(hipMemcpyAsync(w.h_state, w.state, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CG_OK;
}

// Plain float64 CG with the direction update fused into the SpMV (two p
// buffers, A in stencil slices): the SpMV of iteration 0, then per
// iteration k the r update and one launch that ends iteration k (beta, the
// stop test, p_{k+1}, the owed x terms) and runs the SpMV of iteration k+1.
// The polls see the state the separate kernels leave.  With P >= 1 the
// launch carrying the SpMV of every P-th iteration is timed (event slot j:
// the launch queued at step j of a chunk; the last slot pair: iteration 0's).
int plain_fused_loop(cg_handle *h, const PlainWork &w, double *const pbuf[2], int32_t maxit, int P,
                     std::vector<hipEvent_t> &ev, double &t_spmv, int &n_spmv) {
    const int32_t n = h->n;
    hipStream_t st = h->stream;
    const int Gs = h->A.grid, Gv = h->vec_grid;
    const Partials pq{w.part_pq, Gs}, rr{w.part_rr, Gv};
    const Partials setup_rr{w.part_setup, Gs}, setup_bb{w.part_setup + Gs, Gs};
    const int C = h->opts.check_every;
    auto sampled = [P](int32_t it) { return P > 0 && it % P == 0; };
    if (P) {
        ev.resize(2 * (size_t)C + 2);
        for (auto &e : ev)
            if (!e) HIP_TRY(hipEventCreate(&e));
    }
    hipEvent_t *const ev0 = P ? &ev[2 * (size_t)C] : nullptr;
    if (sampled(0)) HIP_TRY(hipEventRecord(ev0[0], st));
    HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, Gs, pbuf[0], w.q, pbuf[0], nullptr, nullptr, w.part_pq,
                        setup_rr, setup_bb, w.state, kSpmvDot, 1, st));
    if (sampled(0)) HIP_TRY(hipEventRecord(ev0[1], st));
    bool first_pending = sampled(0);
    int32_t k = 0;
    bool running = true;
    while (running) {
        const int32_t chunk = maxit == 0 ? 0 : std::min<int32_t>(C, maxit - k);
        for (int32_t j = 0; j < chunk; ++j) {
            const int32_t kk = k + j;
            HIP_TRY(launch_update_r(n, Gv, w.r, w.q, w.part_rr, pq, w.state, kk, st));
            if (sampled(kk + 1)) HIP_TRY(hipEventRecord(ev[2 * j], st));
            HIP_TRY(launch_spmv_dir(h->A.dev(), h->A.sched, Gs, pbuf[kk & 1], w.r, pbuf[(kk + 1) & 1], w.x,
                                    w.q, w.part_pq, rr, no_partials(), w.state, kk, 0, st));
            if (sampled(kk + 1)) HIP_TRY(hipEventRecord(ev[2 * j + 1], st));
        }
        const int32_t it0 = k;
        k += chunk;
        const int rc = work_state_read(h, w);
        if (rc) return rc;
        const DevState &s = *w.h_state;
        running = s.done == kDoneRunning && k < maxit;
        float ms = 0.f;
        if (first_pending) {
            first_pending = false;
            if (fused_spmv_ran(s, 0)) {
                HIP_TRY(hipEventElapsedTime(&ms, ev0[0], ev0[1]));
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
    }
    return CG_OK;
}

int solve_plain(cg_handle *h, const PlainWork &w, const double *b, double *x, double tol, int32_t maxit,
                cg_result *res) {
    const int32_t n = h->n;
    hipStream_t st = h->stream;
    const bool small = h->opts.small_path && n <= small_path_max_rows() &&
                       h->opts.precision == CG_PREC_FP64 && h->opts.precond == CG_PC_NONE &&
                       !h->shared_p();
    if (small) {
        // one launch: x0 read from x, the solution and the true residual
        // written by the kernel, one read-back of the state
        if (h->max_row_len < 0) {
            int32_t L = 0;
            for (int32_t i = 0; i < n; ++i) L = std::max(L, h->A.h_rp[i + 1] - h->A.h_rp[i]);
            h->max_row_len = L;
        }
        // cg_opts.profile: an event pair around the one launch
        struct EventPair {
            hipEvent_t a = nullptr, b = nullptr;
            ~EventPair() {
                if (a) (void)hipEventDestroy(a);
                if (b) (void)hipEventDestroy(b);
            }
        } evp;
        const bool timed = w.events && h->opts.profile > 0 && hipEventCreate(&evp.a) == hipSuccess &&
                           hipEventCreate(&evp.b) == hipSuccess;
        const double t0 = now();
        if (timed) HIP_TRY(hipEventRecord(evp.a, st));
        HIP_TRY(launch_cg_small(n, h->A.d_rp, h->A.d_ci, h->A.d_val, b, x, tol, maxit, w.state,
                                h->max_row_len, st));
        if (timed) HIP_TRY(hipEventRecord(evp.b, st));
        const int rc = work_state_read(h, w);
        if (rc) return rc;
        const DevState &s = *w.h_state;
        const int status = status_of(s.done);
        if (res) {
            res->status = status;
            res->iterations = s.iter;
            res->converged = status == CG_OK;
            res->rel_res_recur = s.bb > 0.0 ? std::sqrt(s.rr) / std::sqrt(s.bb) : 0.0;
            res->rel_res_true = s.bb > 0.0 ? std::sqrt(s.rr_true) / std::sqrt(s.bb) : 0.0;
            res->t_gpu = now() - t0;
            if (timed) {
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, evp.a, evp.b));
                res->t_spmv = 1e-3 * ms;
                res->n_spmv = 1;
            }
        }
        return status;
    }
    HIP_TRY(hipMemcpyAsync(w.x, x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    int rc = work_state_init(h, w, tol, maxit);
    if (rc) return rc;
    double t_gpu = 0.0, t_spmv = 0.0;
    int n_spmv = 0;
    // x updated every other iteration from two p buffers (not with p in
    // shared host memory, whose one buffer the other side reads)
    const bool two_buf = w.p2 != nullptr;
    const bool fused = two_buf && fuse_dir_wanted(h, false) &&
                       spmv_dir_applies(h->A.dev(), h->A.sched, h->A.grid, w.p, w.r, w.p2, w.x, w.q);
    const double t0 = now();
    {
        const int Gs = h->A.grid, Gv = h->vec_grid;
        const Partials setup_rr{w.part_setup, Gs}, setup_bb{w.part_setup + Gs, Gs};
        const Partials pq{w.part_pq, Gs}, rr{w.part_rr, Gv};
        // r = b - A x, p = r (partials of r^T r and b^T b)
        HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, Gs, w.x, w.r, nullptr, b, w.p,
                            w.part_setup, no_partials(), no_partials(), nullptr, kSpmvResidual, 0, st));
        const int C = h->opts.check_every;
        const int P = w.events ? h->opts.profile : 0;   // events around the SpMV of every P-th iteration
        std::vector<hipEvent_t> ev;
        if (P) {
            ev.resize(2 * (size_t)C);
            for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
        }
        auto sampled = [P](int32_t it) { return P > 0 && it % P == 0; };
        double *const pbuf[2] = {w.p, w.p2};
        if (fused) rc = plain_fused_loop(h, w, pbuf, maxit, P, ev, t_spmv, n_spmv);
        int32_t k = 0;
        bool running = !fused;
        while (running) {
            // iteration k = 0 also runs the initial stop test; maxit = 0 runs only that test
            const int32_t chunk = maxit == 0 ? 1 : std::min<int32_t>(C, maxit - k);
            for (int32_t j = 0; j < chunk; ++j) {
                const int32_t kk = k + j;
                if (sampled(kk)) HIP_TRY(hipEventRecord(ev[2 * j], st));
                double *p_k = two_buf ? pbuf[kk & 1] : w.p;
                HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, Gs, p_k, w.q, p_k, nullptr, nullptr,
                                    w.part_pq, setup_rr, setup_bb, w.state, kSpmvDot, kk == 0, st));
                if (sampled(kk)) HIP_TRY(hipEventRecord(ev[2 * j + 1], st));
                if (maxit == 0) break;
                HIP_TRY(launch_update_r(n, Gv, w.r, w.q, w.part_rr, pq, w.state, kk, st));
                if (two_buf) {
                    double *pc = pbuf[kk & 1], *po = pbuf[(kk + 1) & 1];
                    HIP_TRY(launch_update_pxb(n, Gv, w.x, w.r, pc, po, rr, w.state, kk, st));
                } else {
                    HIP_TRY(launch_update_px(n, Gv, w.x, w.r, w.p, rr, w.state, kk, st));
                }
            }
            const int32_t it0 = k;
            k += chunk;
            rc = work_state_read(h, w);
            if (rc) break;
            running = w.h_state->done == kDoneRunning && k < maxit;
            if (P) {
                // time only SpMVs that did work (iterations it0 .. iter, plus a breakdown step)
                int32_t ran = w.h_state->iter - it0 + (w.h_state->done == kDoneBreakdown ? 1 : 0);
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
    }
    t_gpu = now() - t0;
    DevState s = *w.h_state;
    if (s.bb == 0.0) {  // b = 0: the solution is x = 0
        HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * n, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (res) {
            res->status = CG_OK;
            res->iterations = 0;
            res->converged = 1;
        }
        return CG_OK;
    }
    HIP_TRY(hipMemcpyAsync(x, w.x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    // true residual ||b - A x||^2 and ||b||^2 (q as the output scratch)
    HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, h->A.grid, x, w.q, nullptr, b, w.q, w.part_setup,
                        no_partials(), no_partials(), nullptr, kSpmvResidual, 0, st));
    double rr_true = 0.0, bb = 0.0;
    rc = sum_partials_host(h, w.part_setup, h->A.grid, 2, &rr_true, &bb);
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

}  // namespace

static int solve_gpu_only(cg_handle *h, const double *b, double *x, double tol, int32_t maxit,
                          cg_result *res) {
    // x updated every other iteration from two p buffers (not with p in
    // shared host memory, whose one buffer the other side reads)
    const bool two_buf = !h->shared_p();
    if (two_buf && !h->d_p2) {
        const hipError_t e = dmalloc(&h->d_p2, (size_t)h->n + 2);
        if (e != hipSuccess) return fail(CG_ENOMEM, "second p buffer: %s", hipGetErrorString(e));
    }
    const PlainWork w{h->d_x, h->d_r, h->d_q, h->d_p, two_buf ? h->d_p2 : nullptr,
                      h->d_part_setup, h->d_part_pq, h->d_part_rr, h->d_state, h->h_state,
                      true, false};
    return solve_plain(h, w, b, x, tol, maxit, res);
}

// ---------------------------------------------------------------------------
// Mixed precision (GPU-only): float32 inner CG, float64 reliable updates.
// The device runs inner iterations and stops itself when a refinement is due;
// the host then forms the float64 true residual b - A x, decides convergence
// on it, restarts the float32 residual from it and resumes.

static int solve_gpu_mixed(cg_handle *h, const double *b, double *x, double tol, int32_t maxit,
                           cg_result *res) {
    const int32_t n = h->n;
    hipStream_t st = h->stream;
    const int Gs = h->A.grid, Gv = h->vec_grid;
    const Partials pq{h->d_part_pq, Gs}, rrp{h->d_part_rr, Gv};
    const double t0 = now();
    double t_spmv = 0.0;
    int n_spmv = 0;
    int rc = ensure_mixed_vectors(h);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(h->d_x, x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    rc = gpu_state_init(h, tol, maxit);
    if (rc) return rc;
    // float64 true residual r64 = b - A x (into d_r) and its norm
    auto true_residual = [&](double *rr, double *bb) -> int {
        HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, Gs, h->d_x, h->d_r, nullptr, b, h->d_r,
                            h->d_part_setup, no_partials(), no_partials(), nullptr, kSpmvResidual, 0, st));
        return sum_partials_host(h, h->d_part_setup, Gs, 2, rr, bb);
    };
    double rr_true = 0.0, bb = 0.0;
    if ((rc = true_residual(&rr_true, &bb))) return rc;
    int nref = 1;
    if (bb == 0.0) {
        HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * n, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (res) { res->status = CG_OK; res->converged = 1; res->fp64_residuals = nref; }
        return CG_OK;
    }
    const double bnorm = std::sqrt(bb);
    int status = CG_MAXIT, fell_back = 0;
    int32_t k = 0;
    if (std::sqrt(rr_true) < tol * bnorm || rr_true == 0.0) {
        status = CG_OK;
    } else {
        double rho0 = 0.0;
        HIP_TRY(launch_convert_residual(n, Gv, h->d_r, h->d_r32, h->d_p32, h->d_part_rr, 1, st));
        if ((rc = sum_partials_host(h, h->d_part_rr, Gv, 1, &rho0, nullptr))) return rc;
        DevState &S = *h->h_state;
        S.rho[0] = rho0;
        S.bb = bb;
        S.rmax = std::sqrt(rho0);
        S.done = kDoneRunning;
        S.iter = 0;
        HIP_TRY(hipMemcpyAsync(h->d_state, h->h_state, sizeof(DevState), hipMemcpyHostToDevice, st));
        const int C = h->opts.check_every;
        std::vector<hipEvent_t> ev;
        if (h->opts.profile) {
            ev.resize(2 * (size_t)C);
            for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
        }
        const int P = h->opts.profile;   // events around the SpMV of every P-th iteration
        auto sampled = [P](int32_t it) { return P > 0 && it % P == 0; };
        double prev_true = std::sqrt(rr_true);
        int stalls = 0;
        while (k < maxit) {
            const int32_t chunk = std::min<int32_t>(C, maxit - k);
            for (int32_t j = 0; j < chunk; ++j) {
                const int32_t kk = k + j;
                if (sampled(kk)) HIP_TRY(hipEventRecord(ev[2 * j], st));
                HIP_TRY(launch_spmv_f32(h->A.dev(), h->A.sched, Gs, h->d_p32, h->d_q32, h->d_p32,
                                        h->d_part_pq, h->d_state, kSpmvDot, st));
                if (sampled(kk)) HIP_TRY(hipEventRecord(ev[2 * j + 1], st));
                HIP_TRY(launch_update_xr_mixed(n, Gv, h->d_x, h->d_r32, h->d_p32, h->d_q32,
                                               h->d_part_rr, pq, h->d_state, k + j, st));
                HIP_TRY(launch_update_p_mixed(n, Gv, h->d_r32, h->d_p32, rrp, h->d_state, 1, k + j,
                                              0.0, st));
            }
            if ((rc = gpu_state_read(h))) break;
            const int32_t it0 = k;
            k = S.iter;
            if (h->opts.profile) {
                const int32_t ran = std::max(0, std::min<int32_t>(chunk, k - it0 + (S.done == kDoneBreakdown ? 1 : 0)));
                for (int32_t j = 0; j < ran; ++j) {
                    if (!sampled(it0 + j)) continue;
                    float ms = 0.f;
                    HIP_TRY(hipEventElapsedTime(&ms, ev[2 * j], ev[2 * j + 1]));
                    t_spmv += 1e-3 * ms;
                    ++n_spmv;
                }
            }
            if (S.done == kDoneBreakdown) { status = CG_EBREAKDOWN; break; }
            if (S.done == kDoneRefine) {
                // float64 refinement: true residual, its norm, fresh float32 residual
                if ((rc = true_residual(&rr_true, &bb))) break;
                ++nref;
                const double tn = std::sqrt(rr_true);
                if (tn < tol * bnorm || rr_true == 0.0) { status = CG_OK; break; }
                if (k >= maxit) break;
                // stagnation of the float32 inner solve: hand over to float64 CG
                stalls = tn > 0.5 * prev_true ? stalls + 1 : 0;
                prev_true = tn;
                if (stalls >= 3) { fell_back = 1; break; }
                double rho_new = 0.0;
                HIP_TRY(launch_convert_residual(n, Gv, h->d_r, h->d_r32, h->d_p32, h->d_part_rr, 0, st));
                if ((rc = sum_partials_host(h, h->d_part_rr, Gv, 1, &rho_new, nullptr))) break;
                const double beta = rho_new / S.rho[(k - 1) & 1];
                HIP_TRY(launch_update_p_mixed(n, Gv, h->d_r32, h->d_p32, rrp, h->d_state, 0, k, beta, st));
                S.rho[k & 1] = rho_new;
                S.rmax = std::sqrt(rho_new);
                S.done = kDoneRunning;
                HIP_TRY(hipMemcpyAsync(h->d_state, h->h_state, sizeof(DevState), hipMemcpyHostToDevice, st));
                continue;
            }
            if (S.done != kDoneRunning) break;  // iteration limit
        }
        for (auto &e : ev) (void)hipEventDestroy(e);
        if (rc) return rc;
    }
    HIP_TRY(hipMemcpyAsync(x, h->d_x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (fell_back) {
        // finish with float64 CG from the current iterate
        cg_result r64{};
        const int32_t left = std::max(0, maxit - k);
        const int prec = h->opts.precision;
        h->opts.precision = CG_PREC_FP64;
        rc = solve_gpu_only(h, b, x, tol, left, &r64);
        h->opts.precision = prec;
        if (rc < 0) return rc;
        status = rc;
        k += r64.iterations;
        nref += 1;
    }
    double rr_fin = 0.0, bb_fin = 0.0;
    if ((rc = gpu_true_residual(h, b, x, &rr_fin, &bb_fin))) return rc;
    if (res) {
        res->status = status;
        res->iterations = k;
        res->converged = status == CG_OK;
        res->fp64_residuals = nref;
        res->rel_res_recur = std::sqrt(h->h_state->rr) / bnorm;
        res->rel_res_true = std::sqrt(rr_fin) / std::sqrt(bb_fin);
        res->t_gpu = now() - t0;
        res->t_spmv = t_spmv;
        res->n_spmv = n_spmv;
        res->fell_back = fell_back;
    }
    return status;
}

// ---------------------------------------------------------------------------
// split solve: GPU rows [rb, re) and host rows, explicit p exchange

namespace {

struct SplitTimers {
    double gpu = 0, cpu = 0, barrier = 0, d2h = 0, h2d = 0;
    // HIP events around the current GPU phase: gpu sums the kernels' own
    // time, not the time until the host (busy with its rows) looks
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    ~SplitTimers() {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }
};

// Make the updated p visible to both sides (Section 3.4, explicit copy).
int exchange_p(cg_handle *h, SplitTimers &tm) {
    if (h->shared_p()) return CG_OK;   // one copy of p, addressed by both sides
    const int32_t n = h->n, rb = h->rb, re = h->re;
    const bool halo = h->opts.exchange == CG_EXCHANGE_HALO;
    double t0 = now();
    // GPU-owned entries -> host
    if (halo) {
        const int32_t a = (int32_t)h->halo_d2h.size();
        if (a) {
            HIP_TRY(launch_gather(a, h->d_halo_d2h, h->d_p, h->d_pack_d2h, h->stream));
            HIP_TRY(hipMemcpyAsync(h->h_pack_d2h, h->d_pack_d2h, sizeof(double) * a,
                                   hipMemcpyDeviceToHost, h->stream));
            HIP_TRY(hipStreamSynchronize(h->stream));
            for (int32_t i = 0; i < a; ++i) h->h_p[h->halo_d2h[i]] = h->h_pack_d2h[i];
        }
    } else {
        HIP_TRY(hipMemcpyAsync(h->h_p + rb, h->d_p + rb, sizeof(double) * (size_t)(re - rb),
                               hipMemcpyDeviceToHost, h->s_d2h));
        HIP_TRY(hipStreamSynchronize(h->s_d2h));
    }
    double t1 = now();
    tm.d2h += t1 - t0;
    // host-owned entries -> GPU
    if (halo) {
        const int32_t b = (int32_t)h->halo_h2d.size();
        if (b) {
            for (int32_t i = 0; i < b; ++i) h->h_pack_h2d[i] = h->h_p[h->halo_h2d[i]];
            HIP_TRY(hipMemcpyAsync(h->d_pack_h2d, h->h_pack_h2d, sizeof(double) * b,
                                   hipMemcpyHostToDevice, h->stream));
            HIP_TRY(launch_scatter(b, h->d_halo_h2d, h->d_pack_h2d, h->d_p, h->stream));
            HIP_TRY(hipStreamSynchronize(h->stream));
        }
    } else {
        if (rb > 0)
            HIP_TRY(hipMemcpyAsync(h->d_p, h->h_p, sizeof(double) * rb, hipMemcpyHostToDevice, h->s_h2d));
        if (re < n)
            HIP_TRY(hipMemcpyAsync(h->d_p + re, h->h_p + re, sizeof(double) * (size_t)(n - re),
                                   hipMemcpyHostToDevice, h->s_h2d));
        HIP_TRY(hipStreamSynchronize(h->s_h2d));
    }
    tm.h2d += now() - t1;
    return CG_OK;
}

// Wait for the GPU phase bracketed by tm.ev0 / tm.ev1 and add its kernel time.
int wait_gpu(cg_handle *h, SplitTimers &tm) {
    const double t0 = now();
    HIP_TRY(hipStreamSynchronize(h->stream));
    tm.barrier += now() - t0;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, tm.ev0, tm.ev1));
    tm.gpu += 1e-3 * ms;
    return CG_OK;
}

}  // namespace

static int solve_split(cg_handle *h, const double *b, double *x, double tol, int32_t maxit,
                       cg_result *res) {
    const int32_t n = h->n, rb = h->rb, re = h->re, m = h->m;
    const bool gpu = m > 0;
    hipStream_t st = h->stream;
    const int Gs = h->A.grid, Gv = h->vec_grid;
    SplitTimers tm;
    double *hx = h->h_x.data(), *hr = h->h_r.data(), *hq = h->h_q.data(), *hb = h->h_b.data();
    double *hp = h->h_p;
    int rc = CG_OK;
    // host-only handle with host vectors: b and x are read and written in
    // place of device copies (no HIP call in the whole solve)
    const bool host_io = !gpu && h->opts.vectors == CG_VECTORS_HOST;
    // initial transfers: b and x to the host, the GPU block of x to the device buffer
    if (host_io) {
        std::memcpy(hb, b, sizeof(double) * n);
        std::memcpy(hx, x, sizeof(double) * n);
    } else {
        const double t0 = now();
        HIP_TRY(hipMemcpyAsync(hb, b, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hx, x, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        if (gpu) HIP_TRY(hipMemcpyAsync(h->d_x, x + rb, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        tm.d2h += now() - t0;
    }
    if (gpu) {
        HIP_TRY(hipEventCreate(&tm.ev0));
        HIP_TRY(hipEventCreate(&tm.ev1));
        HIP_TRY(hipEventRecord(tm.ev0, st));
        HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, Gs, x, h->d_r, nullptr, b + rb, h->d_p + rb,
                            h->d_part_setup, no_partials(), no_partials(), nullptr, kSpmvResidual, 0, st));
        HIP_TRY(hipEventRecord(tm.ev1, st));
    }
    double t_c = now();
    const double rho_c = host_reduce(h, [&](int32_t i) {
        const double rv = hb[i] - host_row_dot(h, i, hx);
        hr[i] = rv;
        hp[i] = rv;
        return rv * rv;
    });
    const double bb_c = host_reduce(h, [&](int32_t i) { return hb[i] * hb[i]; });
    tm.cpu += now() - t_c;
    double rho = rho_c, bb = bb_c;
    if (gpu) {
        if ((rc = wait_gpu(h, tm))) return rc;
        double rg = 0.0, bg = 0.0;
        if ((rc = sum_partials_host(h, h->d_part_setup, Gs, 2, &rg, &bg))) return rc;
        rho = rg + rho_c;
        bb = bg + bb_c;
        if ((rc = exchange_p(h, tm))) return rc;
    }
    const double bnorm = std::sqrt(bb);
    int status = CG_MAXIT;
    int32_t k = 0;
    if (bnorm == 0.0) {
        if (host_io) {
            std::memset(x, 0, sizeof(double) * n);
        } else {
            HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * n, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        if (res) { res->status = CG_OK; res->converged = 1; }
        return CG_OK;
    }
    for (k = 0; k < maxit; ++k) {
        if (std::sqrt(rho) < tol * bnorm || rho == 0.0) { status = CG_OK; break; }
        // q = A p and p^T q: GPU rows and host rows at the same time
        if (gpu) {
            HIP_TRY(hipEventRecord(tm.ev0, st));
            HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, Gs, h->d_p, h->d_q, h->d_p + rb, nullptr, nullptr,
                                h->d_part_pq, no_partials(), no_partials(), nullptr, kSpmvDot, 0, st));
            HIP_TRY(hipEventRecord(tm.ev1, st));
        }
        t_c = now();
        const double pq_c = host_reduce(h, [&](int32_t i) {
            const double s = host_row_dot(h, i, hp);
            hq[i] = s;
            return hp[i] * s;
        });
        tm.cpu += now() - t_c;
        double pq = pq_c;
        if (gpu) {
            if ((rc = wait_gpu(h, tm))) return rc;
            double pg = 0.0;
            if ((rc = sum_partials_host(h, h->d_part_pq, Gs, 1, &pg, nullptr))) return rc;
            pq = pg + pq_c;
        }
        if (!(pq > 0.0) || !std::isfinite(pq)) { status = CG_EBREAKDOWN; break; }
        const double alpha = rho / pq;
        // x += alpha p, r -= alpha q, r^T r
        if (gpu) {
            HIP_TRY(hipEventRecord(tm.ev0, st));
            HIP_TRY(launch_update_xr(m, Gv, h->d_x, h->d_r, h->d_p + rb, h->d_q, h->d_part_rr,
                                     no_partials(), nullptr, 0, k, alpha, st));
            HIP_TRY(hipEventRecord(tm.ev1, st));
        }
        t_c = now();
        const double rr_c = host_reduce(h, [&](int32_t i) {
            hx[i] = std::fma(alpha, hp[i], hx[i]);
            const double rv = std::fma(-alpha, hq[i], hr[i]);
            hr[i] = rv;
            return rv * rv;
        });
        tm.cpu += now() - t_c;
        double rr = rr_c;
        if (gpu) {
            if ((rc = wait_gpu(h, tm))) return rc;
            double rg = 0.0;
            if ((rc = sum_partials_host(h, h->d_part_rr, Gv, 1, &rg, nullptr))) return rc;
            rr = rg + rr_c;
        }
        const double beta = rr / rho;
        rho = rr;
        if (std::sqrt(rho) < tol * bnorm || rho == 0.0 || k + 1 == maxit) continue;  // p unused
        // p = r + beta p, then exchange
        if (gpu) {
            HIP_TRY(hipEventRecord(tm.ev0, st));
            HIP_TRY(launch_update_p(m, Gv, h->d_r, h->d_p + rb, beta, st));
            HIP_TRY(hipEventRecord(tm.ev1, st));
        }
        t_c = now();
        host_reduce(h, [&](int32_t i) {
            hp[i] = std::fma(beta, hp[i], hr[i]);
            return 0.0;
        });
        tm.cpu += now() - t_c;
        if (gpu) {
            if ((rc = wait_gpu(h, tm))) return rc;
            if ((rc = exchange_p(h, tm))) return rc;
        }
    }
    if (status == CG_MAXIT && (std::sqrt(rho) < tol * bnorm || rho == 0.0)) status = CG_OK;
    // final transfers: host rows of x and the GPU block back into the caller's x
    if (host_io) {
        std::memcpy(x, hx, sizeof(double) * n);
    } else {
        const double t0 = now();
        if (rb > 0) HIP_TRY(hipMemcpyAsync(x, hx, sizeof(double) * rb, hipMemcpyHostToDevice, st));
        if (re < n) HIP_TRY(hipMemcpyAsync(x + re, hx + re, sizeof(double) * (n - re), hipMemcpyHostToDevice, st));
        if (gpu) HIP_TRY(hipMemcpyAsync(x + rb, h->d_x, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        tm.h2d += now() - t0;
    }
    // true residual from the final x (Section 3.1): GPU rows on the GPU, host rows on the host
    if (gpu) HIP_TRY(hipMemcpy(hx + rb, h->d_x, sizeof(double) * m, hipMemcpyDeviceToHost));
    double rr_true = host_reduce(h, [&](int32_t i) {
        const double rv = hb[i] - host_row_dot(h, i, hx);
        return rv * rv;
    });
    if (gpu) {
        double rr_g = 0.0, bb_g = 0.0;
        if ((rc = gpu_true_residual(h, b + rb, x, &rr_g, &bb_g))) return rc;
        rr_true += rr_g;
    }
    if (res) {
        res->status = status;
        res->iterations = k;
        res->converged = status == CG_OK;
        res->rel_res_recur = std::sqrt(rho) / bnorm;
        res->rel_res_true = std::sqrt(rr_true) / bnorm;
        res->t_gpu = tm.gpu;
        res->t_cpu = tm.cpu;
        res->t_barrier = tm.barrier;
        res->t_d2h = tm.d2h;
        res->t_h2d = tm.h2d;
    }
    return status;
}

static_assert(CG_NOALLOC_SCRATCH_BYTES == kScratchBytes, "scratch size in cgmi.h and cgmi_internal.h");

// Plain float64 GPU-only CG with every work buffer in the library's static
// scratch: no device allocation, no pinned host memory, no events.
extern "C" int cg_solve_noalloc(cg_handle *h, const double *b, double *x, double tol, int32_t maxit,
                                cg_result *res) {
    clear_error();
    if (!h) return fail(CG_EINVAL, "handle is NULL");
    if (res) std::memset(res, 0, sizeof *res);
    if (!(tol >= 0.0)) return fail(CG_EINVAL, "tol must be >= 0");
    if (maxit < 0) return fail(CG_EINVAL, "maxit must be >= 0");
    if (h->n > 0 && (!b || !x)) return fail(CG_EINVAL, "b/x is NULL");
    if (!h->gpu_only()) return fail(CG_EINVAL, "cg_solve_noalloc needs a GPU-only handle (rows [0, n))");
    if (h->opts.precision != CG_PREC_FP64 || h->opts.precond != CG_PC_NONE || h->shared_p())
        return fail(CG_EINVAL, "cg_solve_noalloc runs plain float64 CG with p in device memory");
    if (h->opts.vectors != CG_VECTORS_DEVICE)
        return fail(CG_EINVAL, "cg_solve_noalloc takes device vectors (cg_opts.vectors = CG_VECTORS_DEVICE)");
    if (res) {
        res->rows_gpu = h->m;
        res->nnz_gpu = h->nnz_gpu;
    }
    if (h->n == 0) {
        if (res) res->converged = 1;
        return CG_OK;
    }
    if (h->nnz == 0) return fail(CG_EINVAL, "matrix has no nonzeros");
    // carve the scratch: five vectors, three partial arrays, the state
    const size_t vec_bytes = (sizeof(double) * ((size_t)h->n + 2) + 255) & ~size_t(255);
    const size_t part = sizeof(double) * (size_t)h->grid_cap;
    const size_t need = 5 * vec_bytes + 4 * part + ((sizeof(DevState) + 255) & ~size_t(255));
    void *base = nullptr;
    size_t have = 0;
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(scratch_region(h->dev, &base, &have));
    if (need > have) {
        const size_t per_vec = ((have - 4 * part - 256) / 5) & ~size_t(255);
        return fail(CG_EINVAL, "n = %d needs %zu bytes of scratch; the static scratch holds %zu (at most %zu rows)",
                    h->n, need, have, per_vec / sizeof(double) - 2);
    }
    unsigned char *c = static_cast<unsigned char *>(base);
    auto take = [&c](size_t bytes) { unsigned char *r = c; c += bytes; return reinterpret_cast<double *>(r); };
    double *vx = take(vec_bytes), *vr = take(vec_bytes), *vq = take(vec_bytes);
    double *vp = take(vec_bytes), *vp2 = take(vec_bytes);
    double *ps = take(2 * part), *ppq = take(part), *prr = take(part);
    DevState *dst = reinterpret_cast<DevState *>(take(sizeof(DevState)));
    DevState hs{};
    const PlainWork w{vx, vr, vq, vp, vp2, ps, ppq, prr, dst, &hs, false, true};
    const double t0 = now();
    const int rc = solve_plain(h, w, b, x, tol, maxit, res);
    if (res) {
        res->t_solve = now() - t0;
        res->spmv_kind = kind_code(h->A);
        res->rows_gpu = h->m;
        res->nnz_gpu = h->nnz_gpu;
        if (rc < 0 && res->status == 0) res->status = rc;
    }
    return rc;
}

static int solve_impl(cg_handle *h, const double *b, double *x, double tol, int32_t maxit, cg_result *res);

// Host-pointer vectors: device staging buffers of the handle (n float64
// each, allocated on first use).
static int ensure_staging(cg_handle *h) {
    if (h->d_vin) return CG_OK;
    hipError_t e = dmalloc(&h->d_vin, (size_t)h->n);
    if (e == hipSuccess) e = dmalloc(&h->d_vout, (size_t)h->n);
    if (e != hipSuccess) {
        (void)hipFree(h->d_vin);
        h->d_vin = h->d_vout = nullptr;
        return fail(CG_ENOMEM, "staging buffers for host vectors: %s", hipGetErrorString(e));
    }
    return CG_OK;
}

extern "C" int cg_solve(cg_handle *h, const double *b, double *x, double tol, int32_t maxit,
                        cg_result *res) {
    // device vectors, or a host-only handle (its solve reads and writes host
    // vectors directly)
    if (!h || h->opts.vectors != CG_VECTORS_HOST || h->n == 0 || !b || !x || h->m == 0)
        return solve_impl(h, b, x, tol, maxit, res);
    clear_error();
    HIP_TRY(hipSetDevice(h->dev));
    int rc = ensure_staging(h);
    if (rc) return rc;
    const size_t bytes = sizeof(double) * (size_t)h->n;
    const double t0 = now();
    HIP_TRY(hipMemcpyAsync(h->d_vin, b, bytes, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->d_vout, x, bytes, hipMemcpyHostToDevice, h->stream));
    rc = solve_impl(h, h->d_vin, h->d_vout, tol, maxit, res);
    if (rc < 0 && rc != CG_EBREAKDOWN) return rc;
    HIP_TRY(hipMemcpyAsync(x, h->d_vout, bytes, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (res) res->t_solve = now() - t0;   // including the vector copies
    return rc;
}

static int solve_impl(cg_handle *h, const double *b, double *x, double tol, int32_t maxit,
                      cg_result *res) {
    clear_error();
    if (!h) return fail(CG_EINVAL, "handle is NULL");
    if (res) std::memset(res, 0, sizeof *res);
    if (!(tol >= 0.0)) return fail(CG_EINVAL, "tol must be >= 0");
    if (maxit < 0) return fail(CG_EINVAL, "maxit must be >= 0");
    if (h->n > 0 && (!b || !x)) return fail(CG_EINVAL, "b/x is NULL");
    if (res) {
        res->rows_gpu = h->m;
        res->rows_cpu = h->n - h->m;
        res->nnz_gpu = h->nnz_gpu;
        res->nnz_cpu = h->nnz_cpu;
    }
    if (h->n == 0) {
        if (res) res->converged = 1;
        return CG_OK;
    }
    if (!h->nodev) HIP_TRY(hipSetDevice(h->dev));
    const double t0 = now();
    int rc;
    // mapped / managed modes: the solve's p is the shared allocation
    struct PSwap {
        cg_handle *h;
        double *d_p, *h_p;
        ~PSwap() { h->d_p = d_p; h->h_p = h_p; }
    } swap{h, h->d_p, h->h_p};
    if (h->shared_p()) {
        if (h->shared_mode != h->opts.exchange) return fail(CG_EINVAL, "shared p not allocated");
        h->d_p = h->d_pshared + (h->rb & 1);
        h->h_p = h->h_pshared + (h->rb & 1);
    }
    if (h->gpu_only()) {
        if (h->nnz == 0) return fail(CG_EINVAL, "matrix has no nonzeros");
        if (h->opts.precond == CG_PC_FSAI) {
            if (!h->have_factor) return fail(CG_EINVAL, "precond is CG_PC_FSAI but no factor is installed");
            rc = solve_gpu_pcg(h, b, x, tol, maxit, res);
            if (rc == CG_EBREAKDOWN) {
                // preconditioned breakdown (M not SPD in floating point): plain CG from x0
                clear_error();
                if (res) std::memset(res, 0, sizeof *res);
                rc = solve_gpu_only(h, b, x, tol, maxit, res);
                if (res) res->fell_back = 1;
            }
        } else if (h->opts.precision == CG_PREC_MIXED) {
            rc = solve_gpu_mixed(h, b, x, tol, maxit, res);
        } else {
            rc = solve_gpu_only(h, b, x, tol, maxit, res);
        }
    } else {
        rc = solve_split(h, b, x, tol, maxit, res);
    }
    if (res) {
        res->t_solve = now() - t0;
        res->spmv_kind = h->m == 0 ? 0 : kind_code(h->A);
        res->rows_gpu = h->m;
        res->rows_cpu = h->n - h->m;
        res->nnz_gpu = h->nnz_gpu;
        res->nnz_cpu = h->nnz_cpu;
        if (rc < 0 && res->status == 0) res->status = rc;
    }
    if (rc == CG_EBREAKDOWN && !*error_message()) fail(CG_EBREAKDOWN, "breakdown: p^T q <= 0 or not finite");
    return rc;
}

extern "C" int cg_hbm_copy(const double *src, double *dst, int64_t n, void *hip_stream) {
    clear_error();
    if (n < 0) return fail(CG_EINVAL, "n must be >= 0");
    if (n == 0) return CG_OK;
    if (!src || !dst) return fail(CG_EINVAL, "src/dst is NULL");
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(launch_stream_copy(src, dst, n, std::max(8, cus * 16), static_cast<hipStream_t>(hip_stream)));
    return CG_OK;
}

extern "C" int cg_gather(const double *src, const int32_t *idx, double *dst, int64_t n, void *hip_stream) {
    clear_error();
    if (n < 0) return fail(CG_EINVAL, "n must be >= 0");
    if (n == 0) return CG_OK;
    if (!src || !idx || !dst) return fail(CG_EINVAL, "src/idx/dst is NULL");
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t chunks = std::max<int64_t>(1, (n + 2047) / 2048);   // 8 entries per thread
    const int grid = (int)std::min<int64_t>(chunks, (int64_t)std::max(8, cus * 16));
    HIP_TRY(launch_gather_ref(src, idx, dst, n, grid, static_cast<hipStream_t>(hip_stream)));
    return CG_OK;
}

static int spmv_impl(cg_handle *h, const double *x, double *y);

extern "C" int cg_spmv(cg_handle *h, const double *x, double *y) {
    clear_error();
    if (!h) return fail(CG_EINVAL, "handle is NULL");
    if (h->n == 0) return CG_OK;
    if (!x || !y) return fail(CG_EINVAL, "x/y is NULL");
    if (h->opts.vectors != CG_VECTORS_HOST) return spmv_impl(h, x, y);
    if (h->m == 0) {   // host-only handle: every row on host threads, in place
        host_reduce(h, [&](int32_t i) {
            y[i] = host_row_dot(h, i, x);
            return 0.0;
        });
        return CG_OK;
    }
    HIP_TRY(hipSetDevice(h->dev));
    int rc = ensure_staging(h);
    if (rc) return rc;
    const size_t bytes = sizeof(double) * (size_t)h->n;
    HIP_TRY(hipMemcpyAsync(h->d_vin, x, bytes, hipMemcpyHostToDevice, h->stream));
    rc = spmv_impl(h, h->d_vin, h->d_vout);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(y, h->d_vout, bytes, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CG_OK;
}

static int spmv_impl(cg_handle *h, const double *x, double *y) {
    HIP_TRY(hipSetDevice(h->dev));
    const int32_t n = h->n, rb = h->rb, re = h->re, m = h->m;
    if (h->gpu_only()) {
        if (h->nnz == 0) {
            HIP_TRY(hipMemsetAsync(y, 0, sizeof(double) * n, h->stream));
            return CG_OK;
        }
        HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, h->A.grid, x, y, nullptr, nullptr, nullptr, nullptr,
                            no_partials(), no_partials(), nullptr, kSpmvPlain, 0, h->stream));
        return CG_OK;
    }
    // split: GPU rows on the device, host rows from a host copy of x
    double *hx = h->h_x.data(), *hq = h->h_q.data();
    HIP_TRY(hipMemcpyAsync(hx, x, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (m > 0 && h->nnz_gpu > 0)
        HIP_TRY(launch_spmv(h->A.dev(), h->A.sched, h->A.grid, x, y + rb, nullptr, nullptr, nullptr,
                            nullptr, no_partials(), no_partials(), nullptr, kSpmvPlain, 0, h->stream));
    else if (m > 0)
        HIP_TRY(hipMemsetAsync(y + rb, 0, sizeof(double) * m, h->stream));
    host_reduce(h, [&](int32_t i) {
        hq[i] = host_row_dot(h, i, hx);
        return 0.0;
    });
    if (rb > 0) HIP_TRY(hipMemcpyAsync(y, hq, sizeof(double) * rb, hipMemcpyHostToDevice, h->stream));
    if (re < n) HIP_TRY(hipMemcpyAsync(y + re, hq + re, sizeof(double) * (n - re), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CG_OK;
}

extern "C" int cg_spmv_f32(cg_handle *h, const float *x, float *y) {
    clear_error();
    if (!h) return fail(CG_EINVAL, "handle is NULL");
    if (!h->gpu_only() || h->opts.precision != CG_PREC_MIXED || !h->A.d_val32)
        return fail(CG_EINVAL, "cg_spmv_f32 needs a GPU-only handle with mixed precision set");
    if (!x || !y) return fail(CG_EINVAL, "x/y is NULL");
    HIP_TRY(hipSetDevice(h->dev));
    HIP_TRY(launch_spmv_f32(h->A.dev(), h->A.sched, h->A.grid, x, y, nullptr, nullptr, nullptr,
                            kSpmvPlain, h->stream));
    return CG_OK;
}
