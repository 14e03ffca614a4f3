// kernels_small.hip -- the whole of Algorithm 1 for a small system in one
// workgroup of 1024 threads (gfx950).
//
// p lives in LDS (every row may read any entry); thread t owns rows
// t, t + 1024, ... and keeps their x, r, q in registers.  The launch reads x0
// from the caller's x, writes the solution there, recomputes the true
// residual b - A x at the end and leaves every result in the device state,
// so a solve is one launch and one read-back of that state.
#include <hip/hip_runtime.h>
#include <math.h>

#include "cgmi_internal.h"

namespace cgmi {

namespace {

constexpr int kWave = kWaveSize;
constexpr int kSmallThreads = 1024;
constexpr int kSmallWaves = kSmallThreads / kWave;
constexpr int kSmallMaxRpt = 4;  // more rows per thread spill registers at 1024 threads

// One DPP move of a double (both 32-bit halves with the same lane pattern).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum over the wave, the same value in every lane, without LDS: a butterfly
// inside each row of 16 lanes (swap neighbours, swap pairs, mirror the half
// rows, mirror the row) leaves every lane with its row's sum; the four row
// sums are then read as scalars and added in a fixed order.
__device__ __forceinline__ double wave_allsum_dpp(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Every thread gets the workgroup sum after ONE barrier: each wave posts its
// sum, then every thread adds the kSmallWaves posts itself in the same fixed
// order (so all threads hold bitwise the same value and branch alike).
// Consecutive calls alternate between the two halves of red: a wave can only
// overwrite a half after the next call's barrier, which every thread reaches
// after it has read that half.
__device__ __forceinline__ double small_allsum(double v, double (*red)[kSmallWaves], int &half) {
    v = wave_allsum_dpp(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) red[half][w] = v;
    __syncthreads();
    double s = red[half][0];
#pragma unroll
    for (int i = 1; i < kSmallWaves; ++i) s += red[half][i];
    half ^= 1;
    return s;
}

// Row storage of a thread's RPT rows.  W > 0: rows of at most W entries held
// in registers for the whole solve (column indices, below 2^16 here, packed
// two to a register); slots past a row's length hold column = the row itself
// and value 0, which leaves the row's sum unchanged, so the entries are
// summed in CSR order as the CSR variant does.  W == 0: the row bounds in
// registers, columns and values read from memory at every product.
template <int RPT, int W>
struct SmallRows {
    static_assert(kSmallThreads * kSmallMaxRpt <= 65536, "packed 16-bit columns");
    static constexpr int WP = (W + 1) / 2;
    uint32_t colp[RPT][WP];
    double a[RPT][W];
    __device__ void load(int32_t n, const int32_t *rp, const int32_t *ci, const double *val) {
        const int t = threadIdx.x;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int i = t + j * kSmallThreads;
            const int32_t beg = i < n ? rp[i] : 0;
            const int32_t len = i < n ? rp[i + 1] - beg : 0;
            const uint32_t self = i < n ? (uint32_t)i : 0u;
#pragma unroll
            for (int e = 0; e < WP; ++e) colp[j][e] = 0;
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const uint32_t c = e < len ? (uint32_t)ci[beg + e] : self;
                colp[j][e / 2] |= c << (16 * (e & 1));
                a[j][e] = e < len ? val[beg + e] : 0.0;
            }
        }
    }
    template <class Get>
    __device__ __forceinline__ double dot(int j, Get get) const {
        double s = 0.0;
#pragma unroll
        for (int e = 0; e < W; ++e) s = fma(a[j][e], get((colp[j][e / 2] >> (16 * (e & 1))) & 0xFFFFu), s);
        return s;
    }
};

template <int RPT>
struct SmallRows<RPT, 0> {
    int32_t r0[RPT], r1[RPT];
    const int32_t *ci;
    const double *val;
    __device__ void load(int32_t n, const int32_t *rp, const int32_t *ci_, const double *val_) {
        ci = ci_;
        val = val_;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int i = threadIdx.x + j * kSmallThreads;
            r0[j] = i < n ? rp[i] : 0;
            r1[j] = i < n ? rp[i + 1] : 0;
        }
    }
    template <class Get>
    __device__ __forceinline__ double dot(int j, Get get) const {
        double s = 0.0;
        for (int k = r0[j]; k < r1[j]; ++k) s = fma(val[k], get(ci[k]), s);
        return s;
    }
};

template <int RPT, int W>
__global__ __launch_bounds__(kSmallThreads) void k_cg_small(int32_t n, const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            const double *__restrict__ val,
                                                            const double *__restrict__ b,
                                                            double *__restrict__ x, double tol,
                                                            int32_t maxit, DevState *__restrict__ st) {
    extern __shared__ double s_p[];
    __shared__ double red[2][kSmallWaves];
    int half = 0;
    const int t = threadIdx.x;
    SmallRows<RPT, W> A;
    A.load(n, rp, ci, val);
    double xr[RPT], rr[RPT], qq[RPT];
    double acc_r = 0.0, acc_b = 0.0;
    // r = b - A x0, p = r, rho = r^T r, bb = b^T b
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = t + j * kSmallThreads;
        xr[j] = rr[j] = 0.0;
        if (i < n) {
            const double s = A.dot(j, [&](int c) { return x[c]; });
            const double bi = b[i];
            xr[j] = x[i];
            rr[j] = bi - s;
            acc_r = fma(rr[j], rr[j], acc_r);
            acc_b = fma(bi, bi, acc_b);
            s_p[i] = rr[j];
        }
    }
    double rho = small_allsum(acc_r, red, half);
    const double bb = small_allsum(acc_b, red, half);
    if (bb == 0.0) {
        // b = 0: the solution is x = 0
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int i = t + j * kSmallThreads;
            if (i < n) x[i] = 0.0;
        }
        if (t == 0) {
            st->iter = 0;
            st->done = kDoneConverged;
            st->rho[0] = st->rr = st->bb = st->rr_true = 0.0;
        }
        return;
    }
    const double bnorm = sqrt(bb);
    int status = kDoneMaxit;
    int k = 0;
    for (k = 0; k < maxit; ++k) {
        if (sqrt(rho) < tol * bnorm || rho == 0.0) {
            status = kDoneConverged;
            break;
        }
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int i = t + j * kSmallThreads;
            qq[j] = 0.0;
            if (i < n) {
                const double s = A.dot(j, [&](int c) { return s_p[c]; });
                qq[j] = s;
                acc = fma(s_p[i], s, acc);
            }
        }
        const double pq = small_allsum(acc, red, half);
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = kDoneBreakdown;
            break;
        }
        const double alpha = rho / pq;
        acc = 0.0;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int i = t + j * kSmallThreads;
            if (i < n) {
                xr[j] = fma(alpha, s_p[i], xr[j]);
                rr[j] = fma(-alpha, qq[j], rr[j]);
                acc = fma(rr[j], rr[j], acc);
            }
        }
        const double rho_new = small_allsum(acc, red, half);
        const double beta = rho_new / rho;
        rho = rho_new;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int i = t + j * kSmallThreads;
            if (i < n) s_p[i] = fma(beta, s_p[i], rr[j]);
        }
        __syncthreads();
    }
    if (status == kDoneMaxit && (sqrt(rho) < tol * bnorm || rho == 0.0)) status = kDoneConverged;
    // the solution to the caller, and into LDS for the true residual b - A x
    // (every read of p has passed a barrier: the loop top follows one, a
    // breakdown follows the p^T q sum)
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = t + j * kSmallThreads;
        if (i < n) {
            x[i] = xr[j];
            s_p[i] = xr[j];
        }
    }
    __syncthreads();
    double acc_t = 0.0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = t + j * kSmallThreads;
        if (i < n) {
            // rows read once more from memory, so the registers holding them
            // are free after the loop; the same CSR order
            double s = 0.0;
            for (int kk = rp[i]; kk < rp[i + 1]; ++kk) s = fma(val[kk], s_p[ci[kk]], s);
            const double rv = b[i] - s;
            acc_t = fma(rv, rv, acc_t);
        }
    }
    const double rr_true = small_allsum(acc_t, red, half);
    if (t == 0) {
        st->iter = k;
        st->done = status;
        st->rho[0] = rho;
        st->rr = rho;
        st->bb = bb;
        st->rr_true = rr_true;
    }
}

}  // namespace

int small_path_max_rows() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        size_t lds = 64 * 1024;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            lds = prop.sharedMemPerBlock;
        const int by_lds = (int)((lds > 1024 ? lds - 1024 : 0) / sizeof(double));
        cached = by_lds < kSmallThreads * kSmallMaxRpt ? by_lds : kSmallThreads * kSmallMaxRpt;
    }
    return cached;
}

hipError_t launch_cg_small(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
                           const double *b, double *x, double tol, int32_t maxit, DevState *st,
                           int32_t max_row_len, hipStream_t s) {
    if (n <= 0 || n > small_path_max_rows() || max_row_len < 0) return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * (size_t)n;
    const int rpt = (n + kSmallThreads - 1) / kSmallThreads;
    const int L = max_row_len;
#define CGMI_SMALL(R, W)                                                                             \
    hipLaunchKernelGGL((k_cg_small<R, W>), dim3(1), dim3(kSmallThreads), lds, s, n, rp, ci, val, b, x, \
                       tol, maxit, st)
    // register-resident rows where RPT x W entries fit beside the vectors
    if (rpt <= 1 && L <= 8) CGMI_SMALL(1, 8);
    else if (rpt <= 1 && L <= 20) CGMI_SMALL(1, 20);
    else if (rpt <= 2 && L <= 8) CGMI_SMALL(2, 8);
    else if (rpt <= 2 && L <= 12) CGMI_SMALL(2, 12);
    else if (rpt <= 4 && L <= 5) CGMI_SMALL(4, 5);
    else if (rpt <= 1) CGMI_SMALL(1, 0);
    else if (rpt <= 2) CGMI_SMALL(2, 0);
    else CGMI_SMALL(4, 0);
#undef CGMI_SMALL
    return hipGetLastError();
}

}  // namespace cgmi
