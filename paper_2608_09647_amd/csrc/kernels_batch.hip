// kernels_batch.hip -- batched multi-RHS CG in one persistent launch (gfx950).
//
// Each pair (system k, right-hand side j) runs the CG recurrence of
// Algorithm 1 with its own scalars.  A team of workgroups owns the rows of
// system k for the whole launch; lane j of every 16-lane row group handles
// right-hand side j, so the 16 values of one row of a vector form one
// contiguous 128-byte line and a gathered p_c of all right-hand sides is one
// line per column c.
//
// One iteration is three phases separated by team barriers:
//   A: q = A p on the team's rows, partial p^T q per right-hand side;
//   B: alpha = rho / p^T q (team sum), x += alpha p, r -= alpha q, partial r^T r;
//   C: stop test and beta = r^T r / rho (team sum), p = r + beta p.
// Every workgroup of a team sums the team's partials itself in a fixed order,
// so all of them take identical decisions (and results are reproducible for
// a fixed schedule).  A barrier is a counter in device memory: each
// workgroup's waves make their stores visible at device scope (release
// fence), one thread adds 1 and waits until the team's count is reached,
// then the waves invalidate stale cache lines (acquire fence).  A wait is
// bounded by a wall-clock limit; on expiry the error flag ends every team.
#include <hip/hip_runtime.h>
#include <math.h>

#include "batch_internal.h"

namespace cgmi {

namespace {

constexpr int kT = kBatchThreads;
constexpr int kL = kBatchLanes;
constexpr int kRS = kBatchRowsPerStep;
constexpr int kWaves = kT / 64;
enum { kSlotPQ = 0, kSlotRR = 1, kSlotBB = 2, kSlotTrue = 3 };
enum { kStOk = 0, kStMaxit = 1, kStBreakdown = -4 };

struct Shared {
    double red[kWaves][kL];
    double tmp[kT];
    double sum[kL];
    double rho[kL], bb[kL], alpha[kL], beta[kL], rr_last[kL];
    int active[kL], status[kL], iter[kL], zero_b[kL];
    int any;
    int ok;
};

// Partial sum over the workgroup for each right-hand side j (lanes with the
// same j are 16 apart), stored at dst[0..15] by threads 0..15.
__device__ __forceinline__ void wg_partial(double v, double *dst, Shared &S) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane < kL) S.red[wv][lane] = v;
    __syncthreads();
    if (threadIdx.x < kL) {
        double s = S.red[0][threadIdx.x];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) s += S.red[q][threadIdx.x];
        dst[threadIdx.x] = s;
    }
    __syncthreads();   // S.red is reused by the next call
}

// Team sum of one slot for every j, in a fixed order, into S.sum.
__device__ __forceinline__ void team_sum(const BatchArgs &a, int first, int T, int slot, Shared &S) {
    const int j = threadIdx.x & (kL - 1), g = threadIdx.x >> 4;
    double v = 0.0;
    for (int r = g; r < T; r += kT / kL)
        v += a.part[((int64_t)(first + r) * kBatchSlots + slot) * kL + j];
    S.tmp[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < kL) {
        double s = 0.0;
        for (int q = 0; q < kT / kL; ++q) s += S.tmp[q * kL + threadIdx.x];
        S.sum[threadIdx.x] = s;
    }
    __syncthreads();
}

// Barrier of the team of system `sys` (T workgroups).  Returns false when the
// launch is being abandoned (time limit or error flag).
__device__ __forceinline__ bool team_sync(const BatchArgs &a, int sys, int T, int &episode,
                                          Shared &S) {
    ++episode;
    if (T == 1) {
        __syncthreads();
        return true;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __hip_atomic_fetch_add(&a.bar[sys], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int target = episode * T;
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(&a.bar[sys], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            if ((int64_t)(wall_clock64() - t0) > a.timeout_ticks) {
                __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        S.ok = ok;
    }
    __syncthreads();
    __threadfence();
    return S.ok != 0;
}

__device__ __forceinline__ bool stop_test(double rr, double bb, double tol) {
    return sqrt(rr) < tol * sqrt(bb) || rr == 0.0;
}

// sum_k val[k] * v[col[k] * nr + j] for one row, in CSR order, each product
// and sum rounded separately (as the oracle's SpMV).
__device__ __forceinline__ double row_dot(const BatchArgs &a, int64_t row, const double *__restrict__ v,
                                          int nr, int j) {
#pragma clang fp contract(off)
    const int k0 = a.rp[row], k1 = a.rp[row + 1];
    double s = 0.0;
    for (int k = k0; k < k1; ++k) s += a.val[k] * v[(int64_t)a.ci[k] * nr + j];
    return s;
}

template <int U>
__global__ __launch_bounds__(kT) void k_batch_cg(BatchArgs a) {
    __shared__ Shared S;
    const int w = blockIdx.x;
    const int sys = a.wg_sys[w];
    if (sys < 0) return;
    const int T = a.team_size[sys], rank = a.wg_rank[w], first = a.team_first[sys];
    const int64_t off = a.row_off[sys], n = a.row_off[sys + 1] - off;
    const int64_t lo = off + n * rank / T, hi = off + n * (rank + 1) / T;
    const int nr = a.nrhs;
    const int j = threadIdx.x & (kL - 1), rsub = threadIdx.x >> 4;
    const bool lane_on = j < nr;
    double *mypart = a.part + (int64_t)w * kBatchSlots * kL;
    int episode = 0;

    // setup: r = b - A x, p = r; partial r^T r and b^T b
    {
        double arr = 0.0, abb = 0.0;
        if (lane_on)
            for (int64_t r0 = lo; r0 < hi; r0 += kRS * U)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t row = r0 + u * kRS + rsub;
                    if (row < hi) {
                        const double s = row_dot(a, row, a.X, nr, j);
                        const int64_t idx = row * nr + j;
                        const double bv = a.B[idx], rv = bv - s;
                        a.R[idx] = rv;
                        a.P[idx] = rv;
                        arr = fma(rv, rv, arr);
                        abb = fma(bv, bv, abb);
                    }
                }
        wg_partial(arr, mypart + kSlotRR * kL, S);
        wg_partial(abb, mypart + kSlotBB * kL, S);
    }
    if (!team_sync(a, sys, T, episode, S)) return;
    team_sum(a, first, T, kSlotRR, S);
    if (threadIdx.x < kL) S.rr_last[threadIdx.x] = S.sum[threadIdx.x];
    __syncthreads();
    team_sum(a, first, T, kSlotBB, S);
    if (threadIdx.x < kL) {
        const int t = threadIdx.x;
        const double rr = S.rr_last[t], bb = S.sum[t];
        S.rho[t] = rr;
        S.bb[t] = bb;
        S.iter[t] = 0;
        S.zero_b[t] = 0;
        S.active[t] = 0;
        S.status[t] = kStOk;
        if (t < nr) {
            if (bb == 0.0) S.zero_b[t] = 1;
            else if (stop_test(rr, bb, a.tol)) S.status[t] = kStOk;
            else if (a.maxit <= 0) S.status[t] = kStMaxit;
            else S.active[t] = 1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int any = 0;
        for (int t = 0; t < kL; ++t) any |= S.active[t];
        S.any = any;
    }
    __syncthreads();

    for (int k = 0; S.any; ++k) {
        // A: q = A p, partial p^T q
        {
            const bool on = lane_on && S.active[j];
            double acc = 0.0;
            if (on)
                for (int64_t r0 = lo; r0 < hi; r0 += kRS * U)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int64_t row = r0 + u * kRS + rsub;
                        if (row < hi) {
                            const double s = row_dot(a, row, a.P, nr, j);
                            const int64_t idx = row * nr + j;
                            a.Q[idx] = s;
                            acc = fma(a.P[idx], s, acc);
                        }
                    }
            wg_partial(acc, mypart + kSlotPQ * kL, S);
        }
        if (!team_sync(a, sys, T, episode, S)) return;
        team_sum(a, first, T, kSlotPQ, S);
        if (threadIdx.x < kL) {
            const int t = threadIdx.x;
            S.alpha[t] = 0.0;
            if (S.active[t]) {
                const double pq = S.sum[t];
                if (!(pq > 0.0) || !isfinite(pq)) {
                    S.status[t] = kStBreakdown;
                    S.iter[t] = k;
                    S.active[t] = 0;
                } else {
                    S.alpha[t] = S.rho[t] / pq;
                }
            }
        }
        __syncthreads();
        // B: x += alpha p, r -= alpha q, partial r^T r
        {
            const bool on = lane_on && S.active[j];
            const double alpha = S.alpha[j];
            double acc = 0.0;
            if (on)
                for (int64_t r0 = lo; r0 < hi; r0 += kRS * U)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int64_t row = r0 + u * kRS + rsub;
                        if (row < hi) {
                            const int64_t idx = row * nr + j;
                            a.X[idx] = fma(alpha, a.P[idx], a.X[idx]);
                            const double rv = fma(-alpha, a.Q[idx], a.R[idx]);
                            a.R[idx] = rv;
                            acc = fma(rv, rv, acc);
                        }
                    }
            wg_partial(acc, mypart + kSlotRR * kL, S);
        }
        if (!team_sync(a, sys, T, episode, S)) return;
        team_sum(a, first, T, kSlotRR, S);
        if (threadIdx.x < kL) {
            const int t = threadIdx.x;
            S.beta[t] = 0.0;
            if (S.active[t]) {
                const double rr = S.sum[t];
                S.iter[t] = k + 1;
                S.rr_last[t] = rr;
                S.beta[t] = rr / S.rho[t];
                S.rho[t] = rr;
                if (stop_test(rr, S.bb[t], a.tol)) {
                    S.status[t] = kStOk;
                    S.active[t] = 0;
                } else if (k + 1 >= a.maxit) {
                    S.status[t] = kStMaxit;
                    S.active[t] = 0;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int any = 0;
            for (int t = 0; t < kL; ++t) any |= S.active[t];
            S.any = any;
        }
        __syncthreads();
        if (!S.any) break;
        // C: p = r + beta p
        {
            const bool on = lane_on && S.active[j];
            const double beta = S.beta[j];
            if (on)
                for (int64_t r0 = lo; r0 < hi; r0 += kRS * U)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int64_t row = r0 + u * kRS + rsub;
                        if (row < hi) {
                            const int64_t idx = row * nr + j;
                            a.P[idx] = fma(beta, a.P[idx], a.R[idx]);
                        }
                    }
        }
        if (!team_sync(a, sys, T, episode, S)) return;
    }

    // b = 0: the solution is x = 0
    if (lane_on && S.zero_b[j])
        for (int64_t row = lo + rsub; row < hi; row += kRS) a.X[row * nr + j] = 0.0;
    if (!team_sync(a, sys, T, episode, S)) return;
    // true residual ||b - A x||^2
    {
        double acc = 0.0;
        if (lane_on)
            for (int64_t row = lo + rsub; row < hi; row += kRS) {
                const int64_t idx = row * nr + j;
                const double rv = a.B[idx] - row_dot(a, row, a.X, nr, j);
                acc = fma(rv, rv, acc);
            }
        wg_partial(acc, mypart + kSlotTrue * kL, S);
    }
    if (!team_sync(a, sys, T, episode, S)) return;
    team_sum(a, first, T, kSlotTrue, S);
    if (rank == 0) {
        if (threadIdx.x < nr) {
            const int t = threadIdx.x;
            const double bn = sqrt(S.bb[t]);
            BatchOutDev o;
            o.status = S.status[t];
            o.iterations = S.iter[t];
            o.rel_res_recur = S.zero_b[t] ? 0.0 : sqrt(S.rr_last[t]) / bn;
            o.rel_res_true = S.zero_b[t] ? 0.0 : sqrt(S.sum[t]) / bn;
            a.out[(int64_t)sys * nr + t] = o;
        }
        if (threadIdx.x == 0) a.episodes[sys] = episode;
    }
}

}  // namespace

int batch_blocks_per_cu(int rows_per_thread) {
    int nb = 0;
    const hipError_t e = rows_per_thread == 2
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_cg<2>, kT, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_cg<1>, kT, 0);
    return e == hipSuccess ? nb : 0;
}

hipError_t launch_batch_cg(const BatchArgs &a, int grid, int rows_per_thread, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    BatchArgs args = a;
    void *params[] = {&args};
    const void *fn = rows_per_thread == 2 ? reinterpret_cast<const void *>(k_batch_cg<2>)
                                          : reinterpret_cast<const void *>(k_batch_cg<1>);
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kT), params, 0, s);
}

}  // namespace cgmi
