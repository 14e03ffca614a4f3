// Host-side internals shared by the runtime files (built by g++):
// error reporting, device matrices (a CSR block uploaded with its SpMV
// schedule), and the solver handle.
#pragma once
#include <hip/hip_runtime_api.h>

#include <omp.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/cgmi.h"
#include "cgmi_internal.h"

namespace cgmi {

int fail(int code, const char *fmt, ...);
void clear_error();
const char *error_message();
double now();
// Square CSR n x n with int32 indices, strictly increasing columns per row.
int validate_csr(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *val);

// Allocator whose value-less construct leaves trivial elements
// uninitialised, so resize() does not write (and fault in) every page from
// one thread; the large host arrays are then filled by parallel loops
// (par_copy), which also first-touch their pages in parallel.
template <class T, class A = std::allocator<T>>
struct NoInitAlloc : A {
    template <class U>
    struct rebind {
        using other = NoInitAlloc<U, typename std::allocator_traits<A>::template rebind_alloc<U>>;
    };
    using A::A;
    template <class U>
    void construct(U *p) noexcept(std::is_nothrow_default_constructible<U>::value) {
        ::new (static_cast<void *>(p)) U;
    }
    template <class U, class... Args>
    void construct(U *p, Args &&...args) {
        std::allocator_traits<A>::construct(static_cast<A &>(*this), p, std::forward<Args>(args)...);
    }
};
template <class T>
using HostVec = std::vector<T, NoInitAlloc<T>>;

// dst[0, count) = src[0, count) by host threads in contiguous chunks.
template <class T>
void par_copy(T *dst, const T *src, size_t count) {
    constexpr size_t kChunk = size_t(1) << 16;
    const int64_t nchunks = (int64_t)((count + kChunk - 1) / kChunk);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nchunks; ++c) {
        const size_t b = (size_t)c * kChunk, e = std::min(count, b + kChunk);
        std::memcpy(dst + b, src + b, sizeof(T) * (e - b));
    }
}

// a[i] += a[i - 1] for i = 1 .. n (a has n + 1 entries): a running sum by
// host threads over contiguous blocks, then each block shifted by the sum
// of the blocks before it.  Integer sums, so the result is the serial one.
template <class T>
void par_running_sum(T *a, int64_t n) {
    const int nt = omp_get_max_threads();
    if (n < (int64_t(1) << 16) || nt < 2) {
        for (int64_t i = 0; i < n; ++i) a[i + 1] += a[i];
        return;
    }
    std::vector<T> blk((size_t)nt + 1, T(0));
#pragma omp parallel num_threads(nt)
    {
        const int t = omp_get_thread_num(), nth = omp_get_num_threads();
        const int64_t lo = 1 + n * t / nth, hi = 1 + n * (t + 1) / nth;
        T s = T(0);
        for (int64_t i = lo; i < hi; ++i) {
            s += a[i];
            a[i] = s;
        }
        blk[(size_t)t + 1] = s;
#pragma omp barrier
#pragma omp single
        {
            blk[0] = a[0];
            for (int u = 0; u < nth; ++u) blk[(size_t)u + 1] += blk[(size_t)u];
        }
        const T off = blk[(size_t)t];
        for (int64_t i = lo; i < hi; ++i) a[i] += off;
    }
}

template <class T>
hipError_t dmalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * count);
}

#define CGMI_HIP_TRY(expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ::cgmi::fail(CG_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// A block of CSR rows on the device: rebased row pointers, global column
// indices, float64 values (col/val padded by kStreamNnz entries), its SpMV
// schedule, and on demand the sliced copy and float32 copies of the values.
struct DevMatrix {
    int32_t m = 0;
    int64_t nnz = 0;
    int32_t pad_col_base = 0;        // global index of local row 0 (sliced padding)
    HostVec<int32_t> h_rp;           // rebased row pointers (m + 1)
    HostVec<int32_t> h_ci;           // columns (nnz)
    HostVec<double> h_val;           // values (nnz)
    int32_t *d_rp = nullptr, *d_ci = nullptr, *d_rows = nullptr;
    double *d_val = nullptr;
    int32_t *d_sell_off = nullptr, *d_sell_ci = nullptr;
    double *d_sell_val = nullptr;
    size_t sell_slots = 0;
    float *d_val32 = nullptr, *d_sell_val32 = nullptr;
    uint8_t *d_sell_len = nullptr;    // sliced layout: row lengths (ntiles x 64 bytes)
    int32_t *d_tile_row = nullptr;    // adaptive stream tiles: first row of each tile
    uint8_t *d_sell_lenx = nullptr;   // gap-coded slices: length and offset bits per row
    uint16_t *d_sell_gap = nullptr;   //   16-bit column codes, slot-major
    int8_t gap_state = 0;             //   0 unchecked, 1 built, -1 the pattern does not fit
    bool use_gap = false;             //   the float64 paired tiles read them (spmv_kind 7)
    uint32_t *d_sell_idx = nullptr;   // dictionary-sliced layout
    int32_t *d_sell_dict = nullptr;
    int32_t *d_st_off = nullptr, *d_st_offs = nullptr;   // stencil-sliced layout
    uint8_t *d_st_mask = nullptr;
    double *d_st_val = nullptr;
    size_t st_slots = 0;
    std::vector<DevMatrix> blocks;    // column-blocked layout: one CSR per column block
    ColBlocks *cb = nullptr;          //   and their launch operands
    int32_t block_cols = 0;           //   columns per block
    Schedule sched{};
    int grid = 8;
    CsrDev dev() const {
        return CsrDev{m, d_rp, d_ci, d_val, sched.identity ? nullptr : d_rows,
                      d_sell_off, d_sell_ci, d_sell_val, d_val32, d_sell_val32,
                      d_sell_idx, d_sell_dict, pad_col_base, cb,
                      d_st_off, d_st_offs, d_st_mask, d_st_val, d_sell_len, d_tile_row,
                      use_gap ? d_sell_lenx : nullptr, use_gap ? d_sell_gap : nullptr};
    }
};

// Copy the rows (row pointers rebased to start at 0 are computed here from
// the global ones: rp[0..m] with rp[0] possibly > 0) and upload them.  val
// may be null: the values are then zero on the device until their owner
// writes them there (d_val, d_sell_val), and no host copy is kept.
int dm_upload(DevMatrix &M, int32_t m, const int32_t *rp, const int32_t *ci, const double *val,
              int32_t pad_col_base);
// Choose the tiling (kind_opt: cg_opts.spmv_kind; 4 asks for dictionary
// slices, used when every slice has at most 15 distinct column offsets and
// rows of at most kSliceMaxWidth entries, else plain slices; 5 asks for
// column blocks of block_cols columns, 0: kColBlockCols), build the row list,
// the sliced copies or the column blocks, size the grid (0: automatic, a
// multiple of 8 up to grid_cap).
int dm_schedule(DevMatrix &M, int kind_opt, int grid_opt, int cus, int grid_cap, bool need_f32,
                int32_t block_cols = 0);
int dm_ensure_f32(DevMatrix &M);
void dm_free(DevMatrix &M);

}  // namespace cgmi

// Solver handle (C ABI type).
struct cg_handle {
    int dev = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t rb = 0, re = 0, m = 0;
    int64_t nnz_gpu = 0, nnz_cpu = 0;
    cg_opts opts{};
    hipStream_t stream = nullptr;   // caller's stream (or null stream)
    hipStream_t s_d2h = nullptr, s_h2d = nullptr;
    int cus = 256;

    // host copy of the matrix (the host complement uses its rows)
    cgmi::HostVec<int32_t> h_rp, h_ci;
    cgmi::HostVec<double> h_val;

    cgmi::DevMatrix A;               // the GPU row block
    int vec_grid = 0;
    int32_t max_row_len = -1;        // longest row (single-workgroup path; -1: not yet known)

    // device vectors
    double *d_pbuf = nullptr;  // allocation behind d_p
    double *d_p = nullptr;     // full length n, d_p + rb is 16-byte aligned
    double *d_p2 = nullptr;    // GPU-only float64: the second p buffer of the
                               // two-iteration x update (allocated on first use)
    double *d_x = nullptr, *d_r = nullptr, *d_q = nullptr;  // m each
    double *d_vin = nullptr, *d_vout = nullptr;  // n each: staging of host vectors
                                                 // (CG_VECTORS_HOST; on first use)
    double *d_part_setup = nullptr;  // 2 x grid: r^T r, b^T b of the residual kernel
    double *d_part_pq = nullptr;
    double *d_part_rr = nullptr;
    double *d_part_rz = nullptr;
    int grid_cap = 0;
    std::vector<double> h_part;
    cgmi::DevState *d_state = nullptr;
    cgmi::DevState *h_state = nullptr;  // pinned

    // mixed precision vectors
    float *d_r32 = nullptr, *d_p32 = nullptr, *d_q32 = nullptr;

    // preconditioner M^-1 = G^T G
    cgmi::DevMatrix G, GT;
    bool have_factor = false;
    double *d_t = nullptr, *d_z = nullptr;
    double *d_r2 = nullptr;            // second r buffer of the fused x/r + G kernel
    int g_width = 0;                   // G's longest row rounded up to 1, 2, 4, 8 (0: not fused)
    struct FsaiSetup *fsai = nullptr;   // learned-factor workspace (fsai.cpp)

    // split mode
    double *h_p = nullptr;  // pinned, length n (device-less handles: h_p_store)
    std::vector<double> h_p_store;
    bool nodev = false;     // host-only handle created without a HIP device
    std::vector<double> h_x, h_r, h_q, h_b;
    std::vector<int32_t> halo_d2h, halo_h2d;  // global column ids
    int32_t *d_halo_d2h = nullptr, *d_halo_h2d = nullptr;
    double *d_pack_d2h = nullptr, *d_pack_h2d = nullptr;
    double *h_pack_d2h = nullptr, *h_pack_h2d = nullptr;  // pinned

    // p held once where both sides address it (CG_EXCHANGE_MAPPED / _MANAGED):
    // n + 2 doubles; the solve uses offset (rb & 1) so p + rb is 16-byte aligned
    int shared_mode = -1;              // mode the allocation was made for (-1: none)
    double *h_pshared = nullptr;       // host address
    double *d_pshared = nullptr;       // device address of the same memory
    bool shared_p() const {
        return opts.exchange == CG_EXCHANGE_MAPPED || opts.exchange == CG_EXCHANGE_MANAGED;
    }

    bool gpu_only() const { return rb == 0 && re == n && n > 0; }
    bool host_only() const { return m == 0; }
};

namespace cgmi {
// Device-side CG helpers used by the solver variants (cgmi.cpp).
int gpu_state_init(cg_handle *h, double tol, int32_t maxit);
int gpu_state_read(cg_handle *h);
int sum_partials_host(cg_handle *h, const double *d_part, int count, int arrays, double *s0,
                      double *s1);
int gpu_true_residual(cg_handle *h, const double *b_own, const double *x_full, double *rr,
                      double *bb);
inline Partials no_partials() { return Partials{nullptr, 0}; }
// GPU rows up to which CG_FUSE_AUTO fuses the direction update into the
// SpMV (measured on 5- and 7-point systems).  Preconditioned: the separate
// update reads z, p and x and writes p and x every iteration, and the fused
// launch was faster at 1,048,576 rows.  Plain CG (x updated every other
// iteration): faster at 262,144 rows, where launches dominate, slower from
// 884,736 rows on, where the extra gathers of r cost more than the pass
// over p they save.
constexpr int32_t kFuseDirAutoRowsPcg = 1 << 21;
constexpr int32_t kFuseDirAutoRowsCg = 1 << 18;
inline bool fuse_dir_wanted(const cg_handle *h, bool pcg) {
    const int32_t lim = pcg ? kFuseDirAutoRowsPcg : kFuseDirAutoRowsCg;
    return h->opts.fuse_dir == CG_FUSE_ON || (h->opts.fuse_dir == CG_FUSE_AUTO && h->m <= lim);
}
int status_of(int done);
// Preconditioned solve (fsai.cpp); on a breakdown it returns CG_EBREAKDOWN
// with x untouched.
int solve_gpu_pcg(cg_handle *h, const double *b, double *x, double tol, int32_t maxit,
                  cg_result *res);
void fsai_free(cg_handle *h);
}  // namespace cgmi
