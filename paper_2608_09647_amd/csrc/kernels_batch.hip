// kernels_batch.hip -- batched multi-RHS CG in one persistent launch (gfx950).
//
// Each pair (system k, right-hand side j) runs the CG recurrence of
// Algorithm 1 with its own scalars.  A team of workgroups owns the rows of
// system k for the whole launch; lane j of every 16-lane row group handles
// right-hand side j, so the 16 values of one row of a vector form one
// contiguous 128-byte line and a gathered p_c of all right-hand sides is one
// line per column c.
//
// A workgroup works through a list of items, each a (system, rank in its
// team) pair, one after the other: heavy systems get teams of their own,
// while light systems that a single workgroup solves are packed, several to
// a workgroup, so that the grid's work evens out.  The host builds the lists
// (first-fit decreasing on weights n_k^e); an item that belongs to a team of
// more than one workgroup is always its workgroup's only item, so no team
// barrier waits on a workgroup that is still busy with an earlier system.
//
// One iteration is three phases separated by team barriers:
//   A: q = A p on the team's rows, partial p^T q per right-hand side;
//   B: alpha = rho / p^T q (team sum), r -= alpha q, partial r^T r;
//   C: stop test and beta = r^T r / rho (team sum), x += alpha p for every
//      right-hand side updated in B, p = r + beta p for those still running.
// Algorithm 1 updates x with r; x is not read again before C, which reads
// the same p, so the x update is done there and B does not read p.
// Every workgroup of a team sums the team's partials itself in a fixed order,
// so all of them take identical decisions (and results are reproducible for
// a fixed schedule).  A barrier is a counter in device memory: every wave
// makes its stores visible device-wide (device-scope release fence), the
// workgroup synchronises, one thread adds 1 to the team's counter and waits
// until the team's count is reached, and device-scope acquire fences (the
// waiting thread's, then every wave's after a second workgroup barrier)
// drop stale cache lines before the workgroup reads what the team wrote.  A
// wait is bounded by a wall-clock limit; on expiry the error flag ends every
// team.
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
    int upd[kL];   // updated r (and owes the x update) in this iteration's phase B
    int any, any_upd;
    int ok;
};

// Partial sum over the workgroup for each right-hand side: a lane holds V
// consecutive right-hand sides j0 .. j0+V-1 (acc[v] for j0 + v); lanes with
// the same j0 are 16/V apart.  Stored at dst[0..15] by threads 0..15.
template <int V>
__device__ __forceinline__ void wg_partial(const double (&acc)[V], double *dst, Shared &S) {
    constexpr int LPR = kL / V;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double v[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
        v[q] = acc[q];
#pragma unroll
        for (int o = LPR; o < 64; o <<= 1) v[q] += __shfl_xor(v[q], o, 64);
    }
    if (lane < LPR)
#pragma unroll
        for (int q = 0; q < V; ++q) S.red[wv][lane * V + q] = v[q];
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
//
// Memory model: team members sit on different XCDs, whose L2 caches are not
// coherent with each other, so what one workgroup writes must be released at
// agent scope before the counter moves and acquired at agent scope before
// another workgroup reads it.  Every wave issues its own agent-scope release
// fence (its stores are written back past its XCD's L2 and complete before
// the fence returns) before the workgroup barrier, so the one thread that
// moves the counter does so after every wave's release; after the counter
// reaches the team's count, thread 0 issues an agent-scope acquire fence and,
// past the second workgroup barrier, every wave issues its own, so each
// wave's following loads come after its own invalidation of stale lines.
__device__ __forceinline__ bool team_sync(const BatchArgs &a, int sys, int T, int &episode,
                                          Shared &S) {
    ++episode;
    if (T == 1) {
        __syncthreads();
        return true;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
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
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        S.ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return S.ok != 0;
}

__device__ __forceinline__ bool stop_test(double rr, double bb, double tol) {
    return sqrt(rr) < tol * sqrt(bb) || rr == 0.0;
}

// V consecutive float64 values at p[idx] (16-byte aligned when V = 2).
template <int V>
__device__ __forceinline__ void ldv(const double *__restrict__ p, int64_t idx, double (&o)[V]) {
    if constexpr (V == 2) {
        const double2 t = *reinterpret_cast<const double2 *>(p + idx);
        o[0] = t.x;
        o[1] = t.y;
    } else {
        o[0] = p[idx];
    }
}
template <int V>
__device__ __forceinline__ void stv(double *__restrict__ p, int64_t idx, const double (&v)[V]) {
    if constexpr (V == 2) {
        *reinterpret_cast<double2 *>(p + idx) = double2{v[0], v[1]};
    } else {
        p[idx] = v[0];
    }
}

// sum_k val[k] * v[col[k] * nr + j0 + q] for one row and the lane's V
// right-hand sides, in CSR order, each product and sum rounded separately (as
// the oracle's SpMV).  Rows of up to kShort entries load all their columns
// and values first (clamped indices, all independent), then issue all
// gathers, so a row costs two memory round trips instead of one per entry;
// longer rows take a plain loop.
constexpr int kShort = 8;

template <int V>
__device__ __forceinline__ void row_dot(const BatchArgs &a, int64_t row, const double *__restrict__ v,
                                        int nr, int j0, double (&s)[V]) {
#pragma clang fp contract(off)
    const int k0 = a.rp[row], k1 = a.rp[row + 1];
    const int len = k1 - k0;
#pragma unroll
    for (int q = 0; q < V; ++q) s[q] = 0.0;
    if (len <= 0) return;
    if (len <= kShort) {
        int c[kShort];
        double w[kShort], pv[kShort][V];
#pragma unroll
        for (int e = 0; e < kShort; ++e) {
            const int k = k0 + (e < len ? e : 0);
            c[e] = a.ci[k];
            w[e] = a.val[k];
        }
#pragma unroll
        for (int e = 0; e < kShort; ++e) ldv<V>(v, (int64_t)c[e] * nr + j0, pv[e]);
#pragma unroll
        for (int e = 0; e < kShort; ++e)
            if (e < len)
#pragma unroll
                for (int q = 0; q < V; ++q) s[q] += w[e] * pv[e][q];
        return;
    }
    for (int k = k0; k < k1; ++k) {
        double pv[V];
        ldv<V>(v, (int64_t)a.ci[k] * nr + j0, pv);
#pragma unroll
        for (int q = 0; q < V; ++q) s[q] += a.val[k] * pv[q];
    }
}

// Columns and values of a row of at most kPipe entries (clamped: entries
// past the row repeat its first, an empty row reads entry 0).
constexpr int kPipe = 6;

__device__ __forceinline__ void row_cw(const BatchArgs &a, int k0, int len, int (&c)[kPipe],
                                       double (&w)[kPipe]) {
    const int base = len > 0 ? k0 : 0;
#pragma unroll
    for (int e = 0; e < kPipe; ++e) {
        const int k = base + (e < len ? e : 0);
        c[e] = a.ci[k];
        w[e] = a.val[k];
    }
}

// Phase A over the thread's rows lo + rsub, lo + rsub + RS, ...: q = A p and
// the partial p^T q, with three rows in flight (while the current row's
// gathers return, the next row's columns and values and the row pointers of
// the one after are loading), so a row costs about one memory round trip
// instead of three.  Sums as row_dot: CSR order, each product and sum
// rounded; rows longer than kPipe go entry by entry in the same order.
template <int V>
__device__ __forceinline__ void spmv_rows_pipelined(const BatchArgs &a, int64_t lo, int64_t hi, int RS,
                                                    int rsub, int nr, int j0, const bool (&on)[V],
                                                    double (&acc)[V]) {
#pragma clang fp contract(off)
    int64_t row = lo + rsub;
    if (row >= hi) return;
    int k0c = a.rp[row], lenc = a.rp[row + 1] - k0c;
    int cc[kPipe];
    double wc[kPipe];
    row_cw(a, k0c, lenc, cc, wc);
    int k0n = 0, k1n = 0;
    if (row + RS < hi) {
        k0n = a.rp[row + RS];
        k1n = a.rp[row + RS + 1];
    }
    for (; row < hi; row += RS) {
        double pv[kPipe][V], po[V];
#pragma unroll
        for (int e = 0; e < kPipe; ++e) ldv<V>(a.P, (int64_t)cc[e] * nr + j0, pv[e]);
        const int64_t idx = row * nr + j0;
        ldv<V>(a.P, idx, po);
        int cn[kPipe];
        double wn[kPipe];
        row_cw(a, k0n, k1n - k0n, cn, wn);
        int k0nn = 0, k1nn = 0;
        if (row + 2 * RS < hi) {
            k0nn = a.rp[row + 2 * RS];
            k1nn = a.rp[row + 2 * RS + 1];
        }
        double sv[V];
#pragma unroll
        for (int q = 0; q < V; ++q) sv[q] = 0.0;
        if (lenc <= kPipe) {
#pragma unroll
            for (int e = 0; e < kPipe; ++e)
                if (e < lenc)
#pragma unroll
                    for (int q = 0; q < V; ++q) sv[q] += wc[e] * pv[e][q];
        } else {
            for (int k = k0c; k < k0c + lenc; ++k) {
                double g[V];
                ldv<V>(a.P, (int64_t)a.ci[k] * nr + j0, g);
                const double wk = a.val[k];
#pragma unroll
                for (int q = 0; q < V; ++q) sv[q] += wk * g[q];
            }
        }
        stv<V>(a.Q, idx, sv);
#pragma unroll
        for (int q = 0; q < V; ++q)
            if (on[q]) acc[q] = fma(po[q], sv[q], acc[q]);
        k0c = k0n;
        lenc = k1n - k0n;
#pragma unroll
        for (int e = 0; e < kPipe; ++e) {
            cc[e] = cn[e];
            wc[e] = wn[e];
        }
        k0n = k0nn;
        k1n = k1nn;
    }
}

// Phase A in strip order, for systems whose rows form lines of D rows (a
// grid numbered line by line; the host sets D where every column offset is
// either below D/4 or within D/4 of D): the workgroup's rows are visited as
// columns x in [s RS, (s+1) RS) of the lines, strip s after strip s - 1,
// each strip walked down the workgroup's lines.  A row's neighbours in the
// lines above and below are then used within a few steps of each other, so
// the gathered lines of p stay in the L2 of every workgroup at once (in row
// order each workgroup keeps two whole lines in flight, 128 KB at D = 512
// and 16 right-hand sides, more than an XCD's L2 holds for all its
// workgroups).  Rows are summed as in spmv_rows_pipelined, three in flight;
// only the order of the rows in the thread's partial p^T q changes.
template <int V>
__device__ __forceinline__ void spmv_rows_strips(const BatchArgs &a, int64_t off, int64_t lo, int64_t hi, int D,
                                                 int RS, int rsub, int nr, int j0, const bool (&on)[V],
                                                 double (&acc)[V]) {
#pragma clang fp contract(off)
    const int64_t l0 = lo - off, l1 = hi - off;       // local rows [l0, l1)
    if (l1 <= l0) return;
    const int64_t y0 = l0 / D, nlines = (l1 - 1) / D - y0 + 1;
    const int nstrips = (D + RS - 1) / RS;
    const int64_t nsteps = nlines * nstrips;
    // global row of step t, or -1 (a column past the line, or outside [lo, hi))
    auto row_at = [&](int64_t t) -> int64_t {
        if (t >= nsteps) return -1;
        const int64_t strip = t / nlines;
        const int64_t x = strip * RS + rsub;
        const int64_t r = (y0 + (t - strip * nlines)) * D + x;
        return (x < D && r >= l0 && r < l1) ? off + r : -1;
    };
    int64_t row = row_at(0);
    int k0c = 0, lenc = 0;
    if (row >= 0) {
        k0c = a.rp[row];
        lenc = a.rp[row + 1] - k0c;
    }
    int cc[kPipe];
    double wc[kPipe];
    row_cw(a, k0c, lenc, cc, wc);
    int64_t rown = row_at(1);
    int k0n = 0, k1n = 0;
    if (rown >= 0) {
        k0n = a.rp[rown];
        k1n = a.rp[rown + 1];
    }
    for (int64_t t = 0; t < nsteps; ++t) {
        double pv[kPipe][V], po[V];
#pragma unroll
        for (int e = 0; e < kPipe; ++e) ldv<V>(a.P, (int64_t)cc[e] * nr + j0, pv[e]);
        const int64_t idx = (row >= 0 ? row : lo) * nr + j0;
        ldv<V>(a.P, idx, po);
        int cn[kPipe];
        double wn[kPipe];
        row_cw(a, k0n, k1n - k0n, cn, wn);
        const int64_t rownn = row_at(t + 2);
        int k0nn = 0, k1nn = 0;
        if (rownn >= 0) {
            k0nn = a.rp[rownn];
            k1nn = a.rp[rownn + 1];
        }
        double sv[V];
#pragma unroll
        for (int q = 0; q < V; ++q) sv[q] = 0.0;
        if (lenc <= kPipe) {
#pragma unroll
            for (int e = 0; e < kPipe; ++e)
                if (e < lenc)
#pragma unroll
                    for (int q = 0; q < V; ++q) sv[q] += wc[e] * pv[e][q];
        } else {
            for (int k = k0c; k < k0c + lenc; ++k) {
                double g[V];
                ldv<V>(a.P, (int64_t)a.ci[k] * nr + j0, g);
                const double wk = a.val[k];
#pragma unroll
                for (int q = 0; q < V; ++q) sv[q] += wk * g[q];
            }
        }
        if (row >= 0) {
            stv<V>(a.Q, idx, sv);
#pragma unroll
            for (int q = 0; q < V; ++q)
                if (on[q]) acc[q] = fma(po[q], sv[q], acc[q]);
        }
        row = rown;
        rown = rownn;
        k0c = k0n;
        lenc = k1n - k0n;
#pragma unroll
        for (int e = 0; e < kPipe; ++e) {
            cc[e] = cn[e];
            wc[e] = wn[e];
        }
        k0n = k0nn;
        k1n = k1nn;
    }
}

// U: rows a thread advances per step in the setup and the vector phases B
// and C (phase A keeps three rows in flight by itself); V: right-hand sides
// per lane (2 needs an even nrhs and 16-byte aligned vectors).
// One system's solve by this workgroup as member `rank` of its team (the
// whole solve when the team is the workgroup alone).  False when the launch
// is being abandoned (a team wait gave up).
template <int U, int V>
__device__ __forceinline__ bool batch_solve_one(const BatchArgs &a, int sys, int rank, Shared &S) {
    constexpr int LPR = kL / V;          // lanes per row
    constexpr int RS = kT / LPR;         // rows per workgroup step
    const int w = blockIdx.x;
    const int T = a.team_size[sys], first = a.team_first[sys];
    const int64_t off = a.row_off[sys], n = a.row_off[sys + 1] - off;
    const int64_t lo = off + n * rank / T, hi = off + n * (rank + 1) / T;
    const int nr = a.nrhs;
    const int j0 = (threadIdx.x % LPR) * V, rsub = threadIdx.x / LPR;
    const bool lane_on = j0 < nr;
    double *mypart = a.part + (int64_t)w * kBatchSlots * kL;
    int episode = 0;

    // setup: r = b - A x, p = r; partial r^T r and b^T b
    {
        double arr[V], abb[V];
#pragma unroll
        for (int q = 0; q < V; ++q) arr[q] = abb[q] = 0.0;
        if (lane_on)
            for (int64_t r0 = lo; r0 < hi; r0 += RS * U)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t row = r0 + u * RS + rsub;
                    if (row < hi) {
                        double s[V], bv[V], rv[V];
                        row_dot<V>(a, row, a.X, nr, j0, s);
                        const int64_t idx = row * nr + j0;
                        ldv<V>(a.B, idx, bv);
#pragma unroll
                        for (int q = 0; q < V; ++q) {
                            rv[q] = bv[q] - s[q];
                            arr[q] = fma(rv[q], rv[q], arr[q]);
                            abb[q] = fma(bv[q], bv[q], abb[q]);
                        }
                        stv<V>(a.R, idx, rv);
                        stv<V>(a.P, idx, rv);
                    }
                }
        wg_partial<V>(arr, mypart + kSlotRR * kL, S);
        wg_partial<V>(abb, mypart + kSlotBB * kL, S);
    }
    if (!team_sync(a, sys, T, episode, S)) return false;
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
            bool on[V];
            bool any_on = false;
#pragma unroll
            for (int q = 0; q < V; ++q) {
                on[q] = lane_on && S.active[j0 + q];
                any_on |= on[q];
            }
            double acc[V];
#pragma unroll
            for (int q = 0; q < V; ++q) acc[q] = 0.0;
            if (any_on && lane_on) {
                const int D = a.strip[sys];
                if (D > 0)
                    spmv_rows_strips<V>(a, off, lo, hi, D, RS, rsub, nr, j0, on, acc);
                else
                    spmv_rows_pipelined<V>(a, lo, hi, RS, rsub, nr, j0, on, acc);
            }
            wg_partial<V>(acc, mypart + kSlotPQ * kL, S);
        }
        if (!team_sync(a, sys, T, episode, S)) return false;
        team_sum(a, first, T, kSlotPQ, S);
        if (threadIdx.x < kL) {
            const int t = threadIdx.x;
            S.alpha[t] = 0.0;
            S.upd[t] = 0;
            if (S.active[t]) {
                const double pq = S.sum[t];
                if (!(pq > 0.0) || !isfinite(pq)) {
                    S.status[t] = kStBreakdown;
                    S.iter[t] = k;
                    S.active[t] = 0;
                } else {
                    S.alpha[t] = S.rho[t] / pq;
                    S.upd[t] = 1;
                }
            }
        }
        __syncthreads();
        // B: r -= alpha q, partial r^T r
        {
            bool on[V];
            bool any_on = false;
            double alpha[V], acc[V];
#pragma unroll
            for (int q = 0; q < V; ++q) {
                on[q] = lane_on && S.active[j0 + q];
                any_on |= on[q];
                alpha[q] = on[q] ? S.alpha[j0 + q] : 0.0;
                acc[q] = 0.0;
            }
            if (any_on)
                for (int64_t r0 = lo; r0 < hi; r0 += RS * U)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int64_t row = r0 + u * RS + rsub;
                        if (row < hi) {
                            const int64_t idx = row * nr + j0;
                            double qv[V], rv[V];
                            ldv<V>(a.Q, idx, qv);
                            ldv<V>(a.R, idx, rv);
#pragma unroll
                            for (int q = 0; q < V; ++q) {
                                if (on[q]) {
                                    rv[q] = fma(-alpha[q], qv[q], rv[q]);
                                    acc[q] = fma(rv[q], rv[q], acc[q]);
                                }
                            }
                            stv<V>(a.R, idx, rv);
                        }
                    }
            wg_partial<V>(acc, mypart + kSlotRR * kL, S);
        }
        if (!team_sync(a, sys, T, episode, S)) return false;
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
            int any = 0, any_upd = 0;
            for (int t = 0; t < kL; ++t) {
                any |= S.active[t];
                any_upd |= S.upd[t];
            }
            S.any = any;
            S.any_upd = any_upd;
        }
        __syncthreads();
        if (!S.any_upd) break;   // every right-hand side broke down in A: nothing owed
        // C: x += alpha p (right-hand sides updated in B), p = r + beta p (still running)
        {
            bool on[V], up[V];
            bool any_on = false, any_up = false;
            double alpha[V], beta[V];
#pragma unroll
            for (int q = 0; q < V; ++q) {
                on[q] = lane_on && S.active[j0 + q];
                up[q] = lane_on && S.upd[j0 + q];
                any_on |= on[q];
                any_up |= up[q];
                alpha[q] = S.alpha[j0 + q];
                beta[q] = S.beta[j0 + q];
            }
            if (any_up)
                for (int64_t r0 = lo; r0 < hi; r0 += RS * U)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int64_t row = r0 + u * RS + rsub;
                        if (row < hi) {
                            const int64_t idx = row * nr + j0;
                            double pv[V], xv[V], rv[V];
                            ldv<V>(a.P, idx, pv);
                            ldv<V>(a.X, idx, xv);
                            if (any_on) ldv<V>(a.R, idx, rv);
#pragma unroll
                            for (int q = 0; q < V; ++q) {
                                if (up[q]) xv[q] = fma(alpha[q], pv[q], xv[q]);
                                if (on[q]) pv[q] = fma(beta[q], pv[q], rv[q]);
                            }
                            stv<V>(a.X, idx, xv);
                            if (any_on) stv<V>(a.P, idx, pv);
                        }
                    }
        }
        if (!S.any) break;       // the x updates above reach the team at the next barrier
        if (!team_sync(a, sys, T, episode, S)) return false;
    }

    // b = 0: the solution is x = 0
    if (lane_on)
        for (int64_t row = lo + rsub; row < hi; row += RS)
#pragma unroll
            for (int q = 0; q < V; ++q)
                if (S.zero_b[j0 + q]) a.X[row * nr + j0 + q] = 0.0;
    if (!team_sync(a, sys, T, episode, S)) return false;
    // true residual ||b - A x||^2
    {
        double acc[V];
#pragma unroll
        for (int q = 0; q < V; ++q) acc[q] = 0.0;
        if (lane_on)
            for (int64_t row = lo + rsub; row < hi; row += RS) {
                const int64_t idx = row * nr + j0;
                double s[V], bv[V];
                row_dot<V>(a, row, a.X, nr, j0, s);
                ldv<V>(a.B, idx, bv);
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    const double rv = bv[q] - s[q];
                    acc[q] = fma(rv, rv, acc[q]);
                }
            }
        wg_partial<V>(acc, mypart + kSlotTrue * kL, S);
    }
    if (!team_sync(a, sys, T, episode, S)) return false;
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
    return true;
}

// Each workgroup solves its list of systems one after another: a member of a
// team of several workgroups has one, a workgroup hosting small systems
// (teams of one) several, so their rows share workgroups instead of each
// taking one.
template <int U, int V>
__global__ __launch_bounds__(kT) void k_batch_cg(BatchArgs a) {
    __shared__ Shared S;
    const int i0 = __builtin_amdgcn_readfirstlane(a.wg_item[blockIdx.x]);
    const int i1 = __builtin_amdgcn_readfirstlane(a.wg_item[blockIdx.x + 1]);
    for (int it = i0; it < i1; ++it) {
        const int sys = __builtin_amdgcn_readfirstlane(a.item_sys[it]);
        const int rank = __builtin_amdgcn_readfirstlane(a.item_rank[it]);
        if (!batch_solve_one<U, V>(a, sys, rank, S)) return;
        __syncthreads();   // S is set up afresh by the next system
    }
}

template <int U, int V>
int occupancy_of() {
    int nb = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_cg<U, V>, kT, 0) == hipSuccess ? nb : 0;
}

}  // namespace

int batch_blocks_per_cu(int rows_per_thread, int rhs_per_lane) {
    if (rhs_per_lane == 2) return rows_per_thread == 2 ? occupancy_of<2, 2>() : occupancy_of<1, 2>();
    return rows_per_thread == 2 ? occupancy_of<2, 1>() : occupancy_of<1, 1>();
}

hipError_t launch_batch_cg(const BatchArgs &a, int grid, int rows_per_thread, int rhs_per_lane, int cooperative,
                          hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    BatchArgs args = a;
    void *params[] = {&args};
    const void *fn;
    if (rhs_per_lane == 2)
        fn = rows_per_thread == 2 ? reinterpret_cast<const void *>(k_batch_cg<2, 2>)
                                  : reinterpret_cast<const void *>(k_batch_cg<1, 2>);
    else
        fn = rows_per_thread == 2 ? reinterpret_cast<const void *>(k_batch_cg<2, 1>)
                                  : reinterpret_cast<const void *>(k_batch_cg<1, 1>);
    if (cooperative) return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kT), params, 0, s);
    // ordinary launch of a grid the caller has checked to be resident (the
    // team waits give up after their time limit if it were not)
    return hipLaunchKernel(fn, dim3(grid), dim3(kT), params, 0, s);
}

}  // namespace cgmi
