// kernels_cg.hip -- float64 CG hot path for gfx950 (CDNA4, wave64).
//
// SpMV q = A p (Section 3.1) is vector CSR: each row is handled by a group of
// L lanes (L = 1, 2, ..., 64) chosen per row-length class ("bin"); rows longer
// than kHugeRow are handled by a whole workgroup.  Work is split into
// wavefront tiles of up to 64 rows: the wavefront loads the tile's row
// pointers cooperatively (one row per lane, coalesced) and hands each group
// its row bounds by cross-lane shuffles, then every group streams
// consecutive col/val entries of its rows (coalesced) for up to 8 rows at a
// time, so a lane keeps up to 8 independent gathers in flight.  Tiles of one
// wavefront never wait for the other wavefronts of the workgroup.
//
// Scalar reductions (p^T q fused into the SpMV, r^T r fused into the x/r
// update: Section 3.3) never use atomics or cache flushes: each workgroup
// stores its partial sum with a plain store, and the *next* kernel -- whose
// start is ordered after the producer's completion -- reduces the partials in
// workgroup order redundantly in every workgroup.  All workgroups therefore
// derive bit-identical alpha / beta / stop decisions, the results are
// deterministic for a fixed grid, and workgroup 0 records them in DevState
// for the host.
#include <hip/hip_runtime.h>
#include <math.h>

#include "cgmi_internal.h"

namespace cgmi {

namespace {

constexpr int kWave = kWaveSize;
constexpr int kWavesPerBlock = kBlock / kWave;

enum { kFlagCheckDone = 1, kFlagFirstIter = 2 };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    return v;
}

// Sum over the workgroup; the result is valid in thread 0.  sh: NT/64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        s = sh[0];
#pragma unroll
        for (int i = 1; i < NT / kWave; ++i) s += sh[i];
    }
    __syncthreads();
    return s;
}

// Every thread of the workgroup gets the sum.
template <int NT>
__device__ __forceinline__ double block_allsum(double v, double *sh, double *bc) {
    double s = block_sum<NT>(v, sh);
    if (threadIdx.x == 0) *bc = s;
    __syncthreads();
    s = *bc;
    __syncthreads();
    return s;
}

// This thread's share of a producer kernel's partials: entries t, t + kBlock,
// t + 2 kBlock, ... added in that order.  The loads of eight entries are
// issued together, so the sum costs one memory round trip per 8 kBlock
// partials instead of one per entry.
__device__ __forceinline__ double thread_partials(const Partials &P) {
    double v = 0.0;
    for (int base = threadIdx.x; base < P.count; base += 8 * kBlock) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * kBlock;
            t[u] = i < P.count ? P.v[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (base + u * kBlock < P.count) v += t[u];
    }
    return v;
}

// Sum of a producer kernel's partials in a fixed order (same in every workgroup).
__device__ __forceinline__ double reduce_partials(const Partials &P, double *sh, double *bc) {
    return block_allsum<kBlock>(thread_partials(P), sh, bc);
}

// Two such sums with one set of workgroup barriers, each in the order of
// reduce_partials; the loads of both arrays are issued together.
// sh: 2 kBlock/64 doubles; bc: 2 doubles.
__device__ __forceinline__ void reduce_partials2(const Partials &P0, const Partials &P1, double *sh,
                                                 double *bc, double &s0, double &s1) {
    constexpr int NW = kBlock / kWave;
    double a0 = 0.0, a1 = 0.0;
    const int cmax = max(P0.count, P1.count);
    for (int base = threadIdx.x; base < cmax; base += 8 * kBlock) {
        double t0[8], t1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * kBlock;
            t0[u] = i < P0.count ? P0.v[i] : 0.0;
            t1[u] = i < P1.count ? P1.v[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * kBlock;
            if (i < P0.count) a0 += t0[u];
            if (i < P1.count) a1 += t1[u];
        }
    }
    const double v0 = wave_sum(a0);
    const double v1 = wave_sum(a1);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) {
        sh[w] = v0;
        sh[NW + w] = v1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = sh[0], b = sh[NW];
#pragma unroll
        for (int i = 1; i < NW; ++i) {
            a += sh[i];
            b += sh[NW + i];
        }
        bc[0] = a;
        bc[1] = b;
    }
    __syncthreads();
    s0 = bc[0];
    s1 = bc[1];
    __syncthreads();
}

__device__ __forceinline__ bool stop_test(double rho, double bb, double tol) {
    return sqrt(rho) < tol * sqrt(bb) || rho == 0.0;
}

__device__ __forceinline__ bool is_block0_thread0() { return blockIdx.x == 0 && threadIdx.x == 0; }

template <int L, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    return v;  // valid in the group's first lane
}

// T: float64, or float32 for the inner solve of mixed precision.
template <class T>
struct SpmvArgs {
    const T *__restrict__ p;      // gathered vector (full length)
    T *__restrict__ q;            // output rows (local)
    const T *__restrict__ p_own;  // p at the block's own rows (dot)
    const T *__restrict__ b;      // residual mode: right-hand side (local)
    T *__restrict__ p_dst;        // residual mode: copy of r (local)
};

template <class T> __device__ __forceinline__ const T *csr_vals(const CsrDev &A);
template <> __device__ __forceinline__ const double *csr_vals<double>(const CsrDev &A) { return A.val; }
template <> __device__ __forceinline__ const float *csr_vals<float>(const CsrDev &A) { return A.val32; }
template <class T> __device__ __forceinline__ const T *sell_vals(const CsrDev &A);
template <> __device__ __forceinline__ const double *sell_vals<double>(const CsrDev &A) { return A.sell_val; }
template <> __device__ __forceinline__ const float *sell_vals<float>(const CsrDev &A) { return A.sell_val32; }

// Dot contributions and residual norms are always accumulated in float64.
template <int MODE, class T>
__device__ __forceinline__ void emit_row(const SpmvArgs<T> &a, int row, T s, double &acc0,
                                         double &acc1) {
    if (MODE == kSpmvResidual) {
        const T bv = a.b[row];
        const T rv = bv - s;
        a.q[row] = rv;
        a.p_dst[row] = rv;
        acc0 = fma((double)rv, (double)rv, acc0);
        acc1 = fma((double)bv, (double)bv, acc1);
    } else if (MODE == kSpmvAccum) {
        a.q[row] = a.q[row] + s;
    } else {
        a.q[row] = s;
        if (MODE == kSpmvDot) acc0 = fma((double)a.p_own[row], (double)s, acc0);
    }
}

// One wavefront tile: `cnt` (<= 64) rows starting at row-list position pos0,
// L lanes per row, rows_per_group(L) rows per group.
template <int L, int MODE, class T>
__device__ __forceinline__ void spmv_wave_tile(const CsrDev &A, int pos0, int cnt, bool identity,
                                               const SpmvArgs<T> &a, double &acc0, double &acc1) {
    const T *__restrict__ vals = csr_vals<T>(A);
    constexpr int G = kWave / L;
    constexpr int U = rows_per_group(L);
    const int lane = threadIdx.x & (kWave - 1);
    const int gl = lane & (L - 1), g = lane / L;
    // unconditional loads (clamped slot) keep the compiler's load counting exact
    const int slot = pos0 + min(lane, cnt - 1);
    const int row_c = identity ? slot : A.rows[slot];
    int beg_l = A.rp[row_c];
    int end_l = A.rp[row_c + 1];
    int row_l = row_c;
    if (lane >= cnt) {
        row_l = -1;
        end_l = beg_l;
    }
    T sum[U];
    int rowu[U], endu[U], nextu[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = u * G + g;
        const int row = __shfl(row_l, j, kWave);
        const int beg = __shfl(beg_l, j, kWave);
        const int end = __shfl(end_l, j, kWave);
        const int k = beg + gl;
        const bool ok = k < end;
        const int kk = ok ? k : 0;  // entry 0 always holds a valid column
        const int c = A.ci[kk];
        const T v = vals[kk];
        const T pv = a.p[c];
        sum[u] = ok ? v * pv : T(0);
        rowu[u] = row;
        endu[u] = end;
        nextu[u] = k + L;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll 2
        for (int k = nextu[u]; k < endu[u]; k += L) sum[u] = fma(vals[k], a.p[A.ci[k]], sum[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const T s = group_sum<L, T>(sum[u]);
        if (gl == 0 && rowu[u] >= 0) emit_row<MODE, T>(a, rowu[u], s, acc0, acc1);
    }
}

// Wavefront tiles are dealt out per XCD: workgroup b runs on XCD b mod 8, and
// XCD x owns the contiguous tile range [x T8, (x+1) T8), walked in order by
// its wavefronts, so the rows an XCD works on at one time are neighbours
// (shared L2 for the gathered vector).  gridDim.x is a multiple of 8.
struct TileWalk {
    int base, j, stride, end, ntiles;
    __device__ TileWalk(int ntiles_) : ntiles(ntiles_) {
        const int xcd = blockIdx.x & 7;
        const int per = (ntiles_ + 7) >> 3;
        base = xcd * per;
        j = __builtin_amdgcn_readfirstlane((int)(blockIdx.x >> 3) * kWavesPerBlock +
                                           (int)(threadIdx.x / kWave));
        stride = (int)(gridDim.x >> 3) * kWavesPerBlock;
        end = per;
    }
    __device__ int next() {  // tile id, or -1 when done
        if (j >= end) return -1;
        const int t = base + j;
        j += stride;
        return t < ntiles ? t : -1;
    }
};

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stream tiles: tile t covers the rows [tile_row[t], tile_row[t+1]), at most
// 64 rows whose entries span at most kStreamNnz slots counted from the first
// entry rounded down to a multiple of 4, so rows of mixed lengths pack into
// full tiles.  The wavefront loads the tile's entries flat (lane l: slots
// 4l..4l+3 and 256+4l..256+4l+3, 16-byte loads of an int4 of columns and of
// the values: two double pairs, or one float4), keeps 8 gathers in flight per
// lane, parks the products (rounded in T) in its own LDS region, and lane j
// then sums row tile_row[t] + j left to right in T, the row's CSR order;
// accumulate mode adds the sum to q only for rows with entries.  Slots past
// the tile re-read the tile's first group (cached) and are never summed; the
// arrays are padded so no load leaves the allocation.  The loop is
// software-pipelined over the wavefront's tiles, two register sets
// alternating: the loads of tile t+1 are issued while tile t's gathers are in
// flight, and past the last tile the prefetch re-reads the current one.
template <class T>
struct StreamSet {
    int r0, nrows, kb, rb_raw, re_raw;
    int4 c[2];
    T v[8];
};

template <class T>
__device__ __forceinline__ void stream_load(const CsrDev &A, int t, StreamSet<T> &S) {
    const T *__restrict__ vals = csr_vals<T>(A);
    const int lane = threadIdx.x & (kWave - 1);
    S.r0 = __builtin_amdgcn_readfirstlane(A.tile_row[t]);
    S.nrows = __builtin_amdgcn_readfirstlane(A.tile_row[t + 1]) - S.r0;
    const int k0 = A.rp[S.r0];
    const int k1 = A.rp[S.r0 + S.nrows];
    S.kb = k0 & ~3;
    const int span = k1 - S.kb;  // slots used by the tile
    const int i = S.r0 + min(lane, S.nrows - 1);
    S.rb_raw = A.rp[i];
    S.re_raw = A.rp[i + 1];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int sb = 4 * lane + g * 4 * kWave;
        const int k = S.kb + (sb < span ? sb : 0);
        S.c[g] = *reinterpret_cast<const int4 *>(A.ci + k);
        if constexpr (sizeof(T) == 8) {
            const double2 a = *reinterpret_cast<const double2 *>(vals + k);
            const double2 b = *reinterpret_cast<const double2 *>(vals + k + 2);
            S.v[4 * g + 0] = a.x;
            S.v[4 * g + 1] = a.y;
            S.v[4 * g + 2] = b.x;
            S.v[4 * g + 3] = b.y;
        } else {
            const float4 a = *reinterpret_cast<const float4 *>(vals + k);
            S.v[4 * g + 0] = a.x;
            S.v[4 * g + 1] = a.y;
            S.v[4 * g + 2] = a.z;
            S.v[4 * g + 3] = a.w;
        }
    }
}

template <int MODE, class T>
__device__ __forceinline__ void stream_step(const CsrDev &A, const SpmvArgs<T> &a, T *lds,
                                             const StreamSet<T> &S, int tn, StreamSet<T> &N,
                                             double &acc0, double &acc1) {
    const int lane = threadIdx.x & (kWave - 1);
    T pv[8];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        pv[4 * g + 0] = a.p[S.c[g].x];
        pv[4 * g + 1] = a.p[S.c[g].y];
        pv[4 * g + 2] = a.p[S.c[g].z];
        pv[4 * g + 3] = a.p[S.c[g].w];
    }
    stream_load<T>(A, tn, N);
    // products of every slot (slots outside the tile are never read)
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int j = 0; j < 4; ++j) lds[4 * lane + g * 4 * kWave + j] = S.v[4 * g + j] * pv[4 * g + j];
    }
    wave_lds_sync();
    const int rb = S.rb_raw - S.kb, re = S.re_raw - S.kb;
    T s = T(0);
    for (int k = rb; k < re; ++k) s += lds[k];
    if (lane < S.nrows) {
        const int row = S.r0 + lane;
        if (MODE == kSpmvAccum) {
            if (re > rb) a.q[row] = a.q[row] + s;
        } else {
            emit_row<MODE, T>(a, row, s, acc0, acc1);
        }
    }
    wave_lds_sync();
}

template <int MODE, class T>
__device__ __forceinline__ void spmv_stream_wave(const CsrDev &A, TileWalk &walk, const SpmvArgs<T> &a, T *lds,
                                                  double &acc0, double &acc1) {
    int t = walk.next();
    if (t < 0) return;
    StreamSet<T> S0, S1;
    stream_load<T>(A, t, S0);
    for (;;) {
        const int t1 = walk.next();
        stream_step<MODE, T>(A, a, lds, S0, t1 >= 0 ? t1 : t, S1, acc0, acc1);
        if (t1 < 0) break;
        const int t2 = walk.next();
        stream_step<MODE, T>(A, a, lds, S1, t2 >= 0 ? t2 : t1, S0, acc0, acc1);
        if (t2 < 0) break;
        t = t2;
    }
}

// Sliced tiles: lane l owns row r0+l of the 64-row slice; slot j of all 64
// rows is contiguous, so the j-th col/val loads and the j-th gather of the
// wavefront each touch 64 consecutive words (for a stencil, 64 consecutive
// entries of p along one diagonal).  Each lane sums its row left to right
// with rounded products, the oracle's order.  Two pipeline stages alternate
// between register sets: the loads of slice t+1 are issued while slice t's
// gathers are in flight.
template <class T>
struct SliceSet {
    int r0, nrows, off, width, len;
    int c[kSliceMaxWidth];
    T v[kSliceMaxWidth];
};

// GAP: the columns from the gap-coded slices (sell_lenx, sell_gap) and the
// row length from the length byte; rows past the block (last slice) decode
// to the block's last row, a column every lane may gather.
template <class T, bool GAP>
__device__ __forceinline__ void slice_load(const CsrDev &A, int t, SliceSet<T> &S) {
    const T *__restrict__ svals = sell_vals<T>(A);
    const int lane = threadIdx.x & (kWave - 1);
    S.r0 = __builtin_amdgcn_readfirstlane(t * kWave);
    S.nrows = min(kWave, A.m - S.r0);
    S.off = A.sell_off[t];
    S.width = (A.sell_off[t + 1] - S.off) / kWave;
    if constexpr (GAP) {
        const uint32_t lx = A.sell_lenx[(int64_t)S.r0 + lane];
        S.len = lane < S.nrows ? (int)(lx & 0xFu) : 0;
        const int o = (int)(((lx >> 4) << 16) | A.sell_gap[S.off + lane]);
        int cur = A.col_base + S.r0 + lane + ((o ^ 0x80000) - 0x80000);
        S.c[0] = cur;
        S.v[0] = svals[S.off + lane];
#pragma unroll
        for (int j = 1; j < kSliceMaxWidth; ++j) {
            const int k = S.off + (j < S.width ? j : 0) * kWave + lane;
            const int g = (int)A.sell_gap[k];
            if (j < S.len) cur += g + 1;
            S.c[j] = cur;
            S.v[j] = svals[k];
        }
    } else {
        const int i = S.r0 + min(lane, S.nrows - 1);
        S.len = lane < S.nrows ? A.rp[i + 1] - A.rp[i] : 0;
#pragma unroll
        for (int j = 0; j < kSliceMaxWidth; ++j) {
            const int k = S.off + (j < S.width ? j : 0) * kWave + lane;
            S.c[j] = A.sell_ci[k];
            S.v[j] = svals[k];
        }
    }
}

template <int MODE, class T, bool GAP>
__device__ __forceinline__ void slice_step(const CsrDev &A, const SpmvArgs<T> &a,
                                           const SliceSet<T> &S, int tn, SliceSet<T> &N,
                                           double &acc0, double &acc1) {
    const int lane = threadIdx.x & (kWave - 1);
    T pv[kSliceMaxWidth];
#pragma unroll
    for (int j = 0; j < kSliceMaxWidth; ++j) pv[j] = a.p[S.c[j]];
    const int myrow = S.r0 + min(lane, S.nrows - 1);
    T pown = T(0), bv = T(0);
    if (MODE == kSpmvDot) pown = a.p_own[myrow];
    if (MODE == kSpmvResidual) bv = a.b[myrow];
    slice_load<T, GAP>(A, tn, N);
    T s = T(0);
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int j = 0; j < kSliceMaxWidth; ++j)
            if (j < S.len) s = s + S.v[j] * pv[j];  // rounded product, then the sum
    }
    if (lane < S.nrows) {
        if (MODE == kSpmvResidual) {
            const T rv = bv - s;
            a.q[myrow] = rv;
            a.p_dst[myrow] = rv;
            acc0 = fma((double)rv, (double)rv, acc0);
            acc1 = fma((double)bv, (double)bv, acc1);
        } else {
            a.q[myrow] = MODE == kSpmvAccum ? T(a.q[myrow] + s) : s;
            if (MODE == kSpmvDot) acc0 = fma((double)pown, (double)s, acc0);
        }
    }
}

// A slice wider than kSliceMaxWidth: a plain loop over its slots.
template <int MODE, class T>
__device__ __forceinline__ void slice_wide(const CsrDev &A, const SpmvArgs<T> &a, int t,
                                           double &acc0, double &acc1) {
    const T *__restrict__ svals = sell_vals<T>(A);
    const int lane = threadIdx.x & (kWave - 1);
    const int r0 = t * kWave, nrows = min(kWave, A.m - r0);
    const int off = A.sell_off[t];
    const int width = (A.sell_off[t + 1] - off) / kWave;
    const int i = r0 + min(lane, nrows - 1);
    const int len = lane < nrows ? A.rp[i + 1] - A.rp[i] : 0;
    T s = T(0);
    for (int j = 0; j < width; ++j) {
        const int k = off + j * kWave + lane;
        const T pv = a.p[A.sell_ci[k]];
        if (j < len) {
#pragma clang fp contract(off)
            s = s + svals[k] * pv;  // rounded product, then the sum
        }
    }
    if (lane < nrows) emit_row<MODE, T>(a, i, s, acc0, acc1);
}

template <int MODE, class T, bool GAP>
__device__ __forceinline__ void spmv_sliced_wave(const CsrDev &A, TileWalk &walk,
                                                 const SpmvArgs<T> &a, int wide, double &acc0,
                                                 double &acc1) {
    if (wide) {
        for (int t = walk.next(); t >= 0; t = walk.next()) slice_wide<MODE, T>(A, a, t, acc0, acc1);
        return;
    }
    int t = walk.next();
    if (t < 0) return;
    SliceSet<T> S0, S1;
    slice_load<T, GAP>(A, t, S0);
    for (;;) {
        const int t1 = walk.next();
        slice_step<MODE, T, GAP>(A, a, S0, t1 >= 0 ? t1 : t, S1, acc0, acc1);
        if (t1 < 0) break;
        const int t2 = walk.next();
        slice_step<MODE, T, GAP>(A, a, S1, t2 >= 0 ? t2 : t1, S0, acc0, acc1);
        if (t2 < 0) break;
        t = t2;
    }
}

// Dictionary-sliced tiles: as the sliced tiles, but the column of slot j of
// lane l is col_base + row + dict[nibble j]: 4 bits per slot instead of a
// 4-byte column, and no row-pointer loads (padding is a reserved nibble).
// Lanes hold the 16 dictionary entries of the slice in a register (lane d and
// its copies d+16, d+32, d+48 hold entry d) and fetch them with a cross-lane
// permute.  Same row order and rounding as the sliced tiles.
template <class T>
struct DictSet {
    int r0, nrows, off, width;
    uint32_t idx;
    int dict;
    T v[kSliceMaxWidth];
};

// NT: stream the slot values and index words (and store q) nontemporally.
template <class T, bool NT>
__device__ __forceinline__ void dict_load(const CsrDev &A, int t, DictSet<T> &S) {
    const T *__restrict__ svals = sell_vals<T>(A);
    const int lane = threadIdx.x & (kWave - 1);
    S.r0 = __builtin_amdgcn_readfirstlane(t * kWave);
    S.nrows = min(kWave, A.m - S.r0);
    S.off = A.sell_off[t];
    S.width = (A.sell_off[t + 1] - S.off) / kWave;
    const uint32_t *ip = &A.sell_idx[(int64_t)t * kWave + lane];
    S.idx = NT ? __builtin_nontemporal_load(ip) : *ip;
    S.dict = A.sell_dict[t * kDictSize + (lane & (kDictSize - 1))];
#pragma unroll
    for (int j = 0; j < kSliceMaxWidth; ++j) {
        const int k = S.off + (j < S.width ? j : 0) * kWave + lane;
        S.v[j] = NT ? __builtin_nontemporal_load(&svals[k]) : svals[k];
    }
}

template <int MODE, class T, bool NT>
__device__ __forceinline__ void dict_step(const CsrDev &A, const SpmvArgs<T> &a, const DictSet<T> &S,
                                          int tn, DictSet<T> &N, double &acc0, double &acc1) {
    const int lane = threadIdx.x & (kWave - 1);
    const int myrow = S.r0 + min(lane, S.nrows - 1);
    const int gcol = A.col_base + myrow;
    T pv[kSliceMaxWidth];
    uint32_t valid = 0;
#pragma unroll
    for (int j = 0; j < kSliceMaxWidth; ++j) {
        const uint32_t b = (S.idx >> (4 * j)) & 0xFu;
        const int o = __shfl(S.dict, (int)b, kWave);
        valid |= b == kDictPad ? 0u : (1u << j);
        pv[j] = a.p[gcol + o];
    }
    T pown = T(0), bv = T(0);
    if (MODE == kSpmvDot) pown = a.p_own[myrow];
    if (MODE == kSpmvResidual) bv = a.b[myrow];
    dict_load<T, NT>(A, tn, N);
    T s = T(0);
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int j = 0; j < kSliceMaxWidth; ++j)
            if (valid & (1u << j)) s = s + S.v[j] * pv[j];  // rounded product, then the sum
    }
    if (lane < S.nrows) {
        if (MODE == kSpmvResidual) {
            const T rv = bv - s;
            a.q[myrow] = rv;
            a.p_dst[myrow] = rv;
            acc0 = fma((double)rv, (double)rv, acc0);
            acc1 = fma((double)bv, (double)bv, acc1);
        } else {
            if (MODE == kSpmvAccum) a.q[myrow] = T(a.q[myrow] + s);
            else if (NT) __builtin_nontemporal_store(s, &a.q[myrow]);
            else a.q[myrow] = s;
            if (MODE == kSpmvDot) acc0 = fma((double)pown, (double)s, acc0);
        }
    }
}

template <int MODE, class T, bool NT>
__device__ __forceinline__ void spmv_dict_wave(const CsrDev &A, TileWalk &walk, const SpmvArgs<T> &a,
                                               double &acc0, double &acc1) {
    int t = walk.next();
    if (t < 0) return;
    DictSet<T> S0, S1;
    dict_load<T, NT>(A, t, S0);
    for (;;) {
        const int t1 = walk.next();
        dict_step<MODE, T, NT>(A, a, S0, t1 >= 0 ? t1 : t, S1, acc0, acc1);
        if (t1 < 0) break;
        const int t2 = walk.next();
        dict_step<MODE, T, NT>(A, a, S1, t2 >= 0 ? t2 : t1, S0, acc0, acc1);
        if (t2 < 0) break;
        t = t2;
    }
}

// Stencil slices: slot j of a slice holds, for every row of the slice, the
// entry at column row + offs[j], an offset the whole slice shares (scalar
// loads per tile); bit j of the row's mask byte says whether the row has it.
// Slots past the slice's width load nothing (a wave-uniform branch); a slot
// the row lacks gathers the row's own entry of p and is not summed.  Rows are
// summed in CSR order with rounded products (the slots ascend with the
// column), so results are bit-exact against the oracle.  One tile at a time:
// 54 registers, 8 waves per SIMD.  float64 only.
template <int MODE, bool NT>
__device__ __forceinline__ void spmv_sten_wave(const CsrDev &A, TileWalk &walk,
                                               const SpmvArgs<double> &a, double &acc0, double &acc1) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int t = walk.next(); t >= 0; t = walk.next()) {
        const int r0 = __builtin_amdgcn_readfirstlane(t * kWave);
        const int nrows = min(kWave, A.m - r0);
        const int off = A.st_off[t];
        const int width = (A.st_off[t + 1] - off) / kWave;
        int offs[kSliceMaxWidth];
#pragma unroll
        for (int j = 0; j < kSliceMaxWidth; ++j) offs[j] = A.st_offs[t * kSliceMaxWidth + j];
        const int myrow = r0 + min(lane, nrows - 1);
        const int gcol = A.col_base + myrow;
        const uint8_t *mp = &A.st_mask[(int64_t)t * kWave + lane];
        const uint32_t mask = NT ? (uint32_t)__builtin_nontemporal_load(mp) : (uint32_t)*mp;
        // slots past the slice's width (uniform across the wave) load nothing
        double v[kSliceMaxWidth], pv[kSliceMaxWidth];
#pragma unroll
        for (int j = 0; j < kSliceMaxWidth; ++j) {
            v[j] = pv[j] = 0.0;
            if (j < width) {
                const int k = off + j * kWave + lane;
                v[j] = NT ? __builtin_nontemporal_load(&A.st_val[k]) : A.st_val[k];
                pv[j] = a.p[(mask >> j) & 1u ? gcol + offs[j] : gcol];
            }
        }
        double pown = 0.0, bv = 0.0;
        if (MODE == kSpmvDot) pown = a.p_own[myrow];
        if (MODE == kSpmvResidual) bv = a.b[myrow];
        double s = 0.0;
        {
#pragma clang fp contract(off)
#pragma unroll
            for (int j = 0; j < kSliceMaxWidth; ++j)
                if ((mask >> j) & 1u) s = s + v[j] * pv[j];  // rounded product, then the sum
        }
        if (lane < nrows) {
            if (MODE == kSpmvResidual) {
                const double rv = bv - s;
                a.q[myrow] = rv;
                a.p_dst[myrow] = rv;
                acc0 = fma(rv, rv, acc0);
                acc1 = fma(bv, bv, acc1);
            } else {
                if (MODE == kSpmvAccum) a.q[myrow] = a.q[myrow] + s;
                else if (NT) __builtin_nontemporal_store(s, &a.q[myrow]);
                else a.q[myrow] = s;
                if (MODE == kSpmvDot) acc0 = fma(pown, s, acc0);
            }
        }
    }
}

// Stencil slices, two rows per lane: a wave takes the slice pair (2u, 2u+1),
// lanes 0-31 the first slice and 32-63 the second, each lane the row pair
// (2h, 2h+1) of its slice, so values, p_own and q move in 16-byte loads and
// stores.  Each half-wave reads its own slice's offsets; the slot loop runs to
// the wider slice's width (uniform), a half past its own width loads nothing.
// Every row is summed exactly as in spmv_sten_wave; the p^T q partial adds
// the lane's two rows in order.  Plain and dot modes, with q and p_own
// 16-byte aligned (checked by the launcher).
//
// Direction mode (kSpmvDir, k_spmv_dir): a.p holds p_k and the kernel
// multiplies by p_{k+1} = d + beta p_k (d = r, or z = M^-1 r), formed on
// the fly for every gathered column with the fma of the separate direction
// update (so each value is bitwise that kernel's); each lane then writes
// p_{k+1} of its own rows to D.p_oth, applies the owed x update with the
// same fmas as the separate kernels, and adds p_{k+1}^T q for its rows.
// D.p_oth holds p_{k-1} on entry (read for x, own rows only, before the
// same lane overwrites it), so no lane reads what another writes.  The
// lane's two rows read adjacent entries at each slot (the offset is the
// slice's), so one 16-byte gather of p and one of d bring both rows'
// operands (this mode gathers twice as much; single 8-byte gathers made
// it slower); where only one of the rows has the slot, the pair starts one
// entry below that row's column (at 0 for column 0), and where neither
// has it, one below the first row, so the loads stay inside the vectors
// when they have at least two entries (m >= 2, checked by the launcher).
typedef double dbl2v __attribute__((ext_vector_type(2)));

// Two consecutive float64 entries from an 8-byte aligned address (one
// 16-byte load; the hardware takes unaligned vector loads).
__device__ __forceinline__ dbl2v load_pair(const double *p) {
    dbl2v v;
    __builtin_memcpy(&v, p, sizeof v);
    return v;
}

struct DirArgs {
    const double *d;      // r, or z = M^-1 r (gathered and own rows)
    double *p_oth;        // own rows: p_{k-1} in, p_{k+1} out
    double *x;            // own rows
    double beta, alpha, alpha_prev;
    int xmode;            // 0: x untouched; 1: x += alpha p_k; 2: x += alpha_prev p_{k-1}, then alpha p_k
};

// x of one row after iteration k (mode as DirArgs::xmode): the fmas of
// k_update_pxb and k_update_p_pcg.
__device__ __forceinline__ double x_owed(int xmode, double x, double alpha, double pk, double alpha_prev,
                                         double pprev) {
    if (xmode == 2) return fma(alpha, pk, fma(alpha_prev, pprev, x));
    if (xmode == 1) return fma(alpha, pk, x);
    return x;
}

template <int MODE, bool NT>
__device__ __forceinline__ void spmv_sten2_wave(const CsrDev &A, TileWalk &walk, const SpmvArgs<double> &a,
                                                double &acc0, const DirArgs &D) {
    const int lane = threadIdx.x & (kWave - 1);
    const int half = lane >> 5, hl = lane & 31;
    const int nt = (A.m + kWave - 1) / kWave;
    for (int u = walk.next(); u >= 0; u = walk.next()) {
        const int t0 = 2 * u;
        const bool two = t0 + 1 < nt;                 // uniform: the pair has a second slice
        const int t1 = two ? t0 + 1 : t0;
        const int off0 = A.st_off[t0], w0 = (A.st_off[t0 + 1] - off0) / kWave;
        const int off1 = A.st_off[t1], w1 = two ? (A.st_off[t1 + 1] - off1) / kWave : 0;
        const int wmax = max(w0, w1);
        const int ts = half ? t1 : t0;
        const bool mine = !half || two;               // this half has a slice
        const int off = half ? off1 : off0;
        const int width = half ? w1 : w0;
        const int ra = ts * kWave + 2 * hl;           // the lane's rows ra, ra + 1
        const bool va = mine && ra < A.m, vb = mine && ra + 1 < A.m;
        const int rca = min(ra, A.m - 1), rcb = min(ra + 1, A.m - 1);
        const int ga = A.col_base + rca, gb = A.col_base + rcb;
        int offs[kSliceMaxWidth];
#pragma unroll
        for (int j = 0; j < kSliceMaxWidth; ++j) offs[j] = A.st_offs[ts * kSliceMaxWidth + j];
        const uint16_t *mp = reinterpret_cast<const uint16_t *>(&A.st_mask[(int64_t)ts * kWave + 2 * hl]);
        const uint32_t m2 = mine ? (NT ? (uint32_t)__builtin_nontemporal_load(mp) : (uint32_t)*mp) : 0u;
        const uint32_t ma = va ? (m2 & 0xFFu) : 0u, mb = vb ? (m2 >> 8) : 0u;
        double sa = 0.0, sb = 0.0;
        dbl2v v[kSliceMaxWidth];
        double pa[kSliceMaxWidth], pb[kSliceMaxWidth];
#pragma unroll
        for (int j = 0; j < kSliceMaxWidth; ++j) {
            v[j] = dbl2v{0.0, 0.0};
            pa[j] = pb[j] = 0.0;
            if (j < wmax) {
                if (j < width) {
                    const dbl2v *vp = reinterpret_cast<const dbl2v *>(&A.st_val[off + j * kWave + 2 * hl]);
                    v[j] = NT ? __builtin_nontemporal_load(vp) : *vp;
                }
                if (MODE == kSpmvDir) {
                    // the lane's two rows read adjacent columns (offsets are
                    // slice-uniform): one 16-byte gather of p and of d each
                    const bool ha = (ma >> j) & 1u, hb = (mb >> j) & 1u;
                    const int ca = ga + offs[j], cb = gb + offs[j];
                    const int at = ha ? (hb ? ca : max(ca - 1, 0)) : max((hb ? cb : ga) - 1, 0);
                    const dbl2v w = load_pair(&a.p[at]), dv = load_pair(&D.d[at]);
                    const dbl2v pn{fma(D.beta, w.x, dv.x), fma(D.beta, w.y, dv.y)};
                    pa[j] = at == ca ? pn.x : pn.y;
                    pb[j] = at + 1 == cb ? pn.y : pn.x;
                } else {
                    pa[j] = a.p[(ma >> j) & 1u ? ga + offs[j] : ga];
                    pb[j] = a.p[(mb >> j) & 1u ? gb + offs[j] : gb];
                }
            }
        }
        {
#pragma clang fp contract(off)
#pragma unroll
            for (int j = 0; j < kSliceMaxWidth; ++j) {
                if ((ma >> j) & 1u) sa = sa + v[j].x * pa[j];  // rounded product, then the sum
                if ((mb >> j) & 1u) sb = sb + v[j].y * pb[j];
            }
        }
        if (MODE == kSpmvDir && va && vb) {
            const dbl2v pk = *reinterpret_cast<const dbl2v *>(&a.p[ra]);
            const dbl2v dv = *reinterpret_cast<const dbl2v *>(&D.d[ra]);
            dbl2v *po = reinterpret_cast<dbl2v *>(&D.p_oth[ra]);
            if (D.xmode) {
                dbl2v *xp = reinterpret_cast<dbl2v *>(&D.x[ra]);
                const dbl2v pp = D.xmode == 2 ? *po : dbl2v{0.0, 0.0};
                dbl2v xv = *xp;
                xv.x = x_owed(D.xmode, xv.x, D.alpha, pk.x, D.alpha_prev, pp.x);
                xv.y = x_owed(D.xmode, xv.y, D.alpha, pk.y, D.alpha_prev, pp.y);
                *xp = xv;
            }
            const dbl2v pn{fma(D.beta, pk.x, dv.x), fma(D.beta, pk.y, dv.y)};
            *po = pn;
            acc0 = fma(pn.x, sa, acc0);
            acc0 = fma(pn.y, sb, acc0);
            dbl2v qv{sa, sb};
            dbl2v *qp = reinterpret_cast<dbl2v *>(&a.q[ra]);
            if (NT) __builtin_nontemporal_store(qv, qp);
            else *qp = qv;
        } else if (MODE == kSpmvDir && va) {   // the last row of an odd row count
            const double pk = a.p[ra];
            if (D.xmode)
                D.x[ra] = x_owed(D.xmode, D.x[ra], D.alpha, pk, D.alpha_prev, D.xmode == 2 ? D.p_oth[ra] : 0.0);
            const double pn = fma(D.beta, pk, D.d[ra]);
            D.p_oth[ra] = pn;
            acc0 = fma(pn, sa, acc0);
            a.q[ra] = sa;
        } else if (va && vb) {
            if (MODE == kSpmvDot) {
                const dbl2v po = *reinterpret_cast<const dbl2v *>(&a.p_own[ra]);
                acc0 = fma(po.x, sa, acc0);
                acc0 = fma(po.y, sb, acc0);
            }
            dbl2v qv{sa, sb};
            dbl2v *qp = reinterpret_cast<dbl2v *>(&a.q[ra]);
            if (NT) __builtin_nontemporal_store(qv, qp);
            else *qp = qv;
        } else if (va) {   // the last row of an odd row count
            if (MODE == kSpmvDot) acc0 = fma(a.p_own[ra], sa, acc0);
            a.q[ra] = sa;
        }
    }
}

// Sliced tiles, two rows per lane (float64, slices of at most kSliceMaxWidth
// slots, plain and dot modes): a wave takes the slice pair (2u, 2u+1) as
// spmv_sten2_wave does, lanes 0-31 the first slice and 32-63 the second, each
// lane the row pair (2h, 2h+1) of its slice.  Slot j's values move in one
// 16-byte load and its columns in one 8-byte load per lane; each row's length
// comes from one byte per row (no row-pointer loads), so padding slots are
// skipped.  A lane gathers its two rows' slot-j entries, so one gather
// instruction of the wave covers slot j of 128 consecutive rows.  The columns
// of the wave's next slice pair are loaded while the current pair's gathers
// and values are in flight (two register sets alternate, so no register move
// waits on a load), which leaves one memory round trip per pair.  Every row
// is summed left to right with rounded products, as in slice_step (bit-exact
// against the oracle).  NT: the matrix is loaded and q stored nontemporally.
struct Sliced2Geo {
    int off, width, wmax, ra;
    bool va, vb, mine;
    uint32_t l2;   // GAP: the two rows' length bytes, loaded with the columns
};

// GAP: the columns come as 16-bit codes (sell_lenx, sell_gap): one 4-byte
// load of the two rows' codes per slot; slot 0 with the row's offset bits
// gives its first column, and inside the row (slot < its length) each
// further slot advances the column by its code plus one; past it the column
// stays (a padding slot gathers the row's last entry again, never summed).
template <bool NT, bool GAP>
__device__ __forceinline__ void sliced2_cols(const CsrDev &A, int u, Sliced2Geo &G, int2 (&c)[kSliceMaxWidth]) {
    const int lane = threadIdx.x & (kWave - 1);
    const int half = lane >> 5, hl = lane & 31;
    const int nt = (A.m + kWave - 1) / kWave;
    const int t0 = 2 * u;
    const bool two = t0 + 1 < nt;                 // uniform: the pair has a second slice
    const int t1 = two ? t0 + 1 : t0;
    const int off0 = A.sell_off[t0], w0 = (A.sell_off[t0 + 1] - off0) / kWave;
    const int off1 = A.sell_off[t1], w1 = two ? (A.sell_off[t1 + 1] - off1) / kWave : 0;
    G.wmax = max(w0, w1);
    const int ts = half ? t1 : t0;
    G.mine = !half || two;                        // this half has a slice
    G.off = half ? off1 : off0;
    G.width = half ? w1 : w0;
    G.ra = ts * kWave + 2 * hl;                   // the lane's rows ra, ra + 1
    G.va = G.mine && G.ra < A.m;
    G.vb = G.mine && G.ra + 1 < A.m;
    if constexpr (GAP) {
        // a half without a slice reads its partner's (ts == t0) bytes and slot
        // 0 (G.off == off0), discards them and gathers a column every lane may
        const uint16_t *lp = reinterpret_cast<const uint16_t *>(&A.sell_lenx[(int64_t)ts * kWave + 2 * hl]);
        G.l2 = NT ? (uint32_t)__builtin_nontemporal_load(lp) : (uint32_t)*lp;
        const uint32_t *g0p = reinterpret_cast<const uint32_t *>(&A.sell_gap[G.off + 2 * hl]);
        const uint32_t g0 = NT ? __builtin_nontemporal_load(g0p) : *g0p;
        // slot 0: 20-bit two's complement offsets from the rows' global
        // indices, bits 16-19 from the bytes
        const int oa = (int)((((G.l2 >> 4) & 0xFu) << 16) | (g0 & 0xFFFFu));
        const int ob = (int)((((G.l2 >> 12) & 0xFu) << 16) | (g0 >> 16));
        const int ga = A.col_base + min(G.ra, A.m - 1);
        int2 cur = G.mine ? make_int2(A.col_base + G.ra + ((oa ^ 0x80000) - 0x80000),
                                      A.col_base + G.ra + 1 + ((ob ^ 0x80000) - 0x80000))
                          : make_int2(ga, ga);
        c[0] = cur;
        const int la = (int)(G.l2 & 0xFu), lb = (int)((G.l2 >> 8) & 0xFu);
#pragma unroll
        for (int j = 1; j < kSliceMaxWidth; ++j) {
            if (j < G.wmax && j < G.width) {
                const uint32_t *gp = reinterpret_cast<const uint32_t *>(&A.sell_gap[G.off + j * kWave + 2 * hl]);
                const uint32_t g = NT ? __builtin_nontemporal_load(gp) : *gp;
                if (j < la) cur.x += (int)(g & 0xFFFFu) + 1;
                if (j < lb) cur.y += (int)(g >> 16) + 1;
            }
            c[j] = cur;
        }
    } else {
        const int ga = A.col_base + min(G.ra, A.m - 1);   // a column every lane may gather
#pragma unroll
        for (int j = 0; j < kSliceMaxWidth; ++j) {
            c[j] = make_int2(ga, ga);
            if (j < G.wmax && j < G.width) {
                const int2 *cp = reinterpret_cast<const int2 *>(&A.sell_ci[G.off + j * kWave + 2 * hl]);
                c[j] = NT ? make_int2(__builtin_nontemporal_load(&cp->x), __builtin_nontemporal_load(&cp->y)) : *cp;
            }
        }
    }
}

template <int MODE, bool NT, bool GAP>
__device__ __forceinline__ void sliced2_step(const CsrDev &A, const SpmvArgs<double> &a, const Sliced2Geo &G,
                                             const int2 (&c)[kSliceMaxWidth], int un, Sliced2Geo &Gn,
                                             int2 (&cn)[kSliceMaxWidth], double &acc0) {
    const int hl = threadIdx.x & 31;
    dbl2v v[kSliceMaxWidth];
    double pa[kSliceMaxWidth], pb[kSliceMaxWidth];
#pragma unroll
    for (int j = 0; j < kSliceMaxWidth; ++j) {
        v[j] = dbl2v{0.0, 0.0};
        pa[j] = pb[j] = 0.0;
        if (j < G.wmax) {
            pa[j] = a.p[c[j].x];
            pb[j] = a.p[c[j].y];
            if (j < G.width) {
                const dbl2v *vp = reinterpret_cast<const dbl2v *>(&A.sell_val[G.off + j * kWave + 2 * hl]);
                v[j] = NT ? __builtin_nontemporal_load(vp) : *vp;
            }
        }
    }
    uint32_t l2 = G.l2;
    if constexpr (!GAP) {
        const int ts = G.ra & ~(kWave - 1);
        const uint16_t *lp = reinterpret_cast<const uint16_t *>(&A.sell_len[(int64_t)ts + 2 * hl]);
        l2 = G.mine ? (NT ? (uint32_t)__builtin_nontemporal_load(lp) : (uint32_t)*lp) : 0u;
    }
    // the next pair's columns (past the last pair: this pair's again, discarded)
    sliced2_cols<NT, GAP>(A, un, Gn, cn);
    const uint32_t lmask = GAP ? 0xFu : 0xFFu;   // gap-coded: the length is the low nibble
    const int la = G.va ? (int)(l2 & lmask) : 0, lb = G.vb ? (int)((l2 >> 8) & lmask) : 0;
    double sa = 0.0, sb = 0.0;
    {
#pragma clang fp contract(off)
#pragma unroll
        for (int j = 0; j < kSliceMaxWidth; ++j) {
            if (j < la) sa = sa + v[j].x * pa[j];  // rounded product, then the sum
            if (j < lb) sb = sb + v[j].y * pb[j];
        }
    }
    const int ra = G.ra;
    if (G.va && G.vb) {
        if (MODE == kSpmvDot) {
            const dbl2v po = *reinterpret_cast<const dbl2v *>(&a.p_own[ra]);
            acc0 = fma(po.x, sa, acc0);
            acc0 = fma(po.y, sb, acc0);
        }
        dbl2v qv{sa, sb};
        dbl2v *qp = reinterpret_cast<dbl2v *>(&a.q[ra]);
        if (NT) __builtin_nontemporal_store(qv, qp);
        else *qp = qv;
    } else if (G.va) {   // the last row of an odd row count
        if (MODE == kSpmvDot) acc0 = fma(a.p_own[ra], sa, acc0);
        a.q[ra] = sa;
    }
}

template <int MODE, bool NT, bool GAP>
__device__ __forceinline__ void spmv_sliced2_wave(const CsrDev &A, TileWalk &walk, const SpmvArgs<double> &a,
                                                  double &acc0) {
    int u = walk.next();
    if (u < 0) return;
    Sliced2Geo G0, G1;
    int2 c0[kSliceMaxWidth], c1[kSliceMaxWidth];
    sliced2_cols<NT, GAP>(A, u, G0, c0);
    for (;;) {
        const int u1 = walk.next();
        sliced2_step<MODE, NT, GAP>(A, a, G0, c0, u1 >= 0 ? u1 : u, G1, c1, acc0);
        if (u1 < 0) break;
        const int u2 = walk.next();
        sliced2_step<MODE, NT, GAP>(A, a, G1, c1, u2 >= 0 ? u2 : u1, G0, c0, acc0);
        if (u2 < 0) break;
        u = u2;
    }
}

// A row longer than kHugeRow: all threads of the workgroup on it.
template <int MODE, class T>
__device__ __forceinline__ void spmv_row_wg(const CsrDev &A, int pos, bool identity,
                                            const SpmvArgs<T> &a, double &acc0, double &acc1,
                                            double *sh) {
    const T *__restrict__ vals = csr_vals<T>(A);
    const int row = identity ? pos : A.rows[pos];
    const int beg = A.rp[row], end = A.rp[row + 1];
    double v = 0.0;  // a long row is reduced in float64 whatever T is
#pragma unroll 4
    for (int k = beg + (int)threadIdx.x; k < end; k += kBlock)
        v = fma((double)vals[k], (double)a.p[A.ci[k]], v);
    const double s = block_sum<kBlock>(v, sh);
    if (threadIdx.x == 0) emit_row<MODE, T>(a, row, (T)s, acc0, acc1);
}

// TILE > 0: one bin of TILE lanes per row in natural row order;
// TILE == 0: binned rows (any order); TILE == -1: stream tiles;
// TILE == -2: sliced tiles of width <= kSliceMaxWidth; -3: wider slices;
// TILE == -4: dictionary-sliced tiles; -5: the same with the matrix streamed
// nontemporally (matrices larger than the last-level cache can hold);
// -6 / -7: stencil slices, cached / nontemporal (float64 only); -8 / -9: the
// same with two rows per lane and 16-byte accesses (plain and dot modes);
// -10 / -11: sliced tiles with two rows per lane, cached / nontemporal
// (float64, plain and dot modes); -12 / -13: the same with gap-coded columns;
// -14: sliced tiles (one row per lane) with gap-coded columns.
template <int MODE, int TILE, class T>
__global__ __launch_bounds__(kBlock) void k_spmv(int32_t m, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci,
                                                 const T *__restrict__ val,
                                                 const int32_t *__restrict__ rows,
                                                 const int32_t *__restrict__ sell_off,
                                                 const int32_t *__restrict__ sell_ci,
                                                 const T *__restrict__ sell_val,
                                                 const uint32_t *__restrict__ sell_idx,
                                                 const int32_t *__restrict__ sell_dict, int32_t col_base,
                                                 const int32_t *__restrict__ st_off,
                                                 const int32_t *__restrict__ st_offs,
                                                 const uint8_t *__restrict__ st_mask,
                                                 const double *__restrict__ st_val,
                                                 const uint8_t *__restrict__ sell_len,
                                                 const int32_t *__restrict__ tile_row,
                                                 const uint8_t *__restrict__ sell_lenx,
                                                 const uint16_t *__restrict__ sell_gap,
                                                 Schedule S, SpmvArgs<T> a, double *__restrict__ out,
                                                 Partials in0, Partials in1,
                                                 DevState *__restrict__ st, int flags) {
    CsrDev A{m, rp, ci, nullptr, rows, sell_off, sell_ci, nullptr, nullptr, nullptr,
             sell_idx, sell_dict, col_base, nullptr, st_off, st_offs, st_mask, st_val, sell_len, tile_row,
             sell_lenx, sell_gap};
    if constexpr (sizeof(T) == 8) {
        A.val = reinterpret_cast<const double *>(val);
        A.sell_val = reinterpret_cast<const double *>(sell_val);
    } else {
        A.val32 = reinterpret_cast<const float *>(val);
        A.sell_val32 = reinterpret_cast<const float *>(sell_val);
    }
    __shared__ double sh[kWavesPerBlock];
    __shared__ double bc;
    __shared__ T s_prod[TILE == -1 ? kWavesPerBlock * kStreamNnz : 1];
    if (flags & kFlagCheckDone) {
        if (st->done) return;
        if (flags & kFlagFirstIter) {
            // stop test at the top of iteration 0 from the setup partials
            const double rr = reduce_partials(in0, sh, &bc);
            const double bb = reduce_partials(in1, sh, &bc);
            const bool conv = stop_test(rr, bb, st->tol);
            const bool stop = conv || st->maxit <= 0;
            if (is_block0_thread0()) {
                st->rho[0] = rr;
                st->rr = rr;
                st->bb = bb;
                if (stop) st->done = conv ? kDoneConverged : kDoneMaxit;
            }
            if (stop) return;
        }
    }
    double acc0 = 0.0, acc1 = 0.0;
    const bool identity = S.identity != 0;
    TileWalk walk(TILE <= -8 && TILE >= -13 ? (S.ntiles + 1) / 2 : S.ntiles);   // slice pairs
    if constexpr (TILE == -2 || TILE == -3) {
        spmv_sliced_wave<MODE, T, false>(A, walk, a, TILE == -3, acc0, acc1);
    } else if constexpr (TILE == -14) {
        spmv_sliced_wave<MODE, T, true>(A, walk, a, 0, acc0, acc1);
    } else if constexpr (TILE == -4 || TILE == -5) {
        spmv_dict_wave<MODE, T, TILE == -5>(A, walk, a, acc0, acc1);
    } else if constexpr (TILE == -6 || TILE == -7) {
        if constexpr (sizeof(T) == 8) spmv_sten_wave<MODE, TILE == -7>(A, walk, a, acc0, acc1);
    } else if constexpr (TILE == -8 || TILE == -9) {
        if constexpr (sizeof(T) == 8 && (MODE == kSpmvPlain || MODE == kSpmvDot))
            spmv_sten2_wave<MODE, TILE == -9>(A, walk, a, acc0, DirArgs{});
    } else if constexpr (TILE <= -10 && TILE >= -13) {
        if constexpr (sizeof(T) == 8 && (MODE == kSpmvPlain || MODE == kSpmvDot))
            spmv_sliced2_wave<MODE, TILE == -11 || TILE == -13, TILE <= -12>(A, walk, a, acc0);
    } else if constexpr (TILE == -1) {
        T *lds = s_prod + (threadIdx.x / kWave) * kStreamNnz;
        spmv_stream_wave<MODE, T>(A, walk, a, lds, acc0, acc1);
    } else if constexpr (TILE > 0) {
        constexpr int L = TILE > 0 ? TILE : 1;
        constexpr int RW = rows_per_wave_tile(L);
        for (int t = walk.next(); t >= 0; t = walk.next()) {
            const int pos0 = t * RW;
            spmv_wave_tile<L, MODE, T>(A, pos0, min(RW, A.m - pos0), true, a, acc0, acc1);
        }
    } else {
        for (int t = walk.next(); t >= 0; t = walk.next()) {
            int bi = 0;
            while (bi + 1 < S.nbins && t >= S.bins[bi + 1].tile_begin) ++bi;
            const Bin B = S.bins[bi];
            const int rw = rows_per_wave_tile(B.lanes);
            const int pos0 = B.first + (t - B.tile_begin) * rw;
            const int cnt = min(rw, B.first + B.count - pos0);
            switch (B.lanes) {
                case 1: spmv_wave_tile<1, MODE, T>(A, pos0, cnt, identity, a, acc0, acc1); break;
                case 2: spmv_wave_tile<2, MODE, T>(A, pos0, cnt, identity, a, acc0, acc1); break;
                case 4: spmv_wave_tile<4, MODE, T>(A, pos0, cnt, identity, a, acc0, acc1); break;
                case 8: spmv_wave_tile<8, MODE, T>(A, pos0, cnt, identity, a, acc0, acc1); break;
                case 16: spmv_wave_tile<16, MODE, T>(A, pos0, cnt, identity, a, acc0, acc1); break;
                case 32: spmv_wave_tile<32, MODE, T>(A, pos0, cnt, identity, a, acc0, acc1); break;
                default: spmv_wave_tile<64, MODE, T>(A, pos0, cnt, identity, a, acc0, acc1); break;
            }
        }
        for (int hrow = blockIdx.x; hrow < S.huge_count; hrow += gridDim.x)
            spmv_row_wg<MODE, T>(A, S.huge_first + hrow, identity, a, acc0, acc1, sh);
    }
    if (MODE == kSpmvPlain || MODE == kSpmvAccum) return;
    const double s0 = block_sum<kBlock>(acc0, sh);
    double s1 = 0.0;
    if (MODE == kSpmvResidual) s1 = block_sum<kBlock>(acc1, sh);
    if (threadIdx.x == 0) {
        out[blockIdx.x] = s0;
        if (MODE == kSpmvResidual) out[gridDim.x + blockIdx.x] = s1;
    }
}

// Column-blocked SpMV, first and last kernels.  Start: the early exit and
// first-iteration stop test of k_spmv, then q = 0.  Finish: the mode's
// epilogue on the accumulated q = A p (p^T q partials, or the residual
// b - A p with its partial sums), one partial per workgroup in row order.
template <class T>
__global__ __launch_bounds__(kBlock) void k_blocked_start(int32_t m, T *__restrict__ q, Partials in0,
                                                          Partials in1, DevState *__restrict__ st,
                                                          int flags) {
    __shared__ double sh[kWavesPerBlock];
    __shared__ double bc;
    if (flags & kFlagCheckDone) {
        if (st->done) return;
        if (flags & kFlagFirstIter) {
            const double rr = reduce_partials(in0, sh, &bc);
            const double bb = reduce_partials(in1, sh, &bc);
            const bool conv = stop_test(rr, bb, st->tol);
            const bool stop = conv || st->maxit <= 0;
            if (is_block0_thread0()) {
                st->rho[0] = rr;
                st->rr = rr;
                st->bb = bb;
                if (stop) st->done = conv ? kDoneConverged : kDoneMaxit;
            }
            if (stop) return;
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock)
        q[i] = T(0);
}

template <int MODE, class T>
__global__ __launch_bounds__(kBlock) void k_blocked_finish(int32_t m, SpmvArgs<T> a, double *__restrict__ out,
                                                           DevState *__restrict__ st, int flags) {
    __shared__ double sh[kWavesPerBlock];
    if ((flags & kFlagCheckDone) && st->done) return;
    double acc0 = 0.0, acc1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock) {
        const T s = a.q[i];
        if (MODE == kSpmvResidual) {
            const T bv = a.b[i];
            const T rv = bv - s;
            a.q[i] = rv;
            a.p_dst[i] = rv;
            acc0 = fma((double)rv, (double)rv, acc0);
            acc1 = fma((double)bv, (double)bv, acc1);
        } else {
            acc0 = fma((double)a.p_own[i], (double)s, acc0);
        }
    }
    const double s0 = block_sum<kBlock>(acc0, sh);
    double s1 = 0.0;
    if (MODE == kSpmvResidual) s1 = block_sum<kBlock>(acc1, sh);
    if (threadIdx.x == 0) {
        out[blockIdx.x] = s0;
        if (MODE == kSpmvResidual) out[gridDim.x + blockIdx.x] = s1;
    }
}

// Preconditioned CG: the r update fused with t = G r_new (G of at most W
// entries per row, CSR; W = 1, 2, 4 or 8).  Thread per row: r_new = r - alpha q
// for the row (into the other r buffer, so neighbours still read r), and
// t_i = sum_k G_ik r_new_k with r_new_k formed on the fly by the same fma as
// its owner (identical bits), summed in CSR order with rounded products;
// partial r_new^T r_new per workgroup.  alpha and the breakdown test as in
// k_update_xr.  x += alpha p is left to k_update_p_pcg, which reads p anyway.
template <int W>
__global__ __launch_bounds__(kBlock) void k_pcg_xr_g(int32_t m, const int32_t *__restrict__ grp,
                                                     const int32_t *__restrict__ gci,
                                                     const double *__restrict__ gval,
                                                     const double *__restrict__ r_old, double *__restrict__ r_new,
                                                     const double *__restrict__ q,
                                                     double *__restrict__ t, double *__restrict__ out,
                                                     Partials pq_in, DevState *__restrict__ st, int32_t k) {
    __shared__ double sh[kWavesPerBlock];
    __shared__ double bc;
    if (st->done) return;
    const double pq = reduce_partials(pq_in, sh, &bc);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (is_block0_thread0()) {
            st->pq = pq;
            st->iter = k;
            st->done = kDoneBreakdown;
        }
        return;
    }
    const double alpha = st->rho[k & 1] / pq;
    if (is_block0_thread0()) {
        st->pq = pq;
        st->r_iter = k + 1;
    }
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock) {
        const double rv = fma(-alpha, q[i], r_old[i]);
        r_new[i] = rv;
        acc = fma(rv, rv, acc);
        const int k0 = grp[i], len = grp[i + 1] - k0;
        int c[W];
        double w[W], rn[W];
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const int kk = k0 + (e < len ? e : 0);
            c[e] = gci[kk];
            w[e] = gval[kk];
        }
#pragma unroll
        for (int e = 0; e < W; ++e) rn[e] = fma(-alpha, q[c[e]], r_old[c[e]]);
        double s = 0.0;
        {
#pragma clang fp contract(off)
#pragma unroll
            for (int e = 0; e < W; ++e)
                if (e < len) s = s + w[e] * rn[e];
        }
        t[i] = s;
    }
    const double s = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// The same with G in stencil slices (the layout of spmv_sten_wave): a
// wavefront takes a 64-row slice, lane l row r0 + l; the columns of slot j are
// the rows plus the slice's j-th offset, so no column index is loaded and all
// gathers of a row issue at once.  Slots ascend with the column and absent
// ones are skipped, so t_i is summed exactly as by k_pcg_xr_g.
__global__ __launch_bounds__(kBlock) void k_pcg_xr_gs(int32_t m, const int32_t *__restrict__ st_off,
                                                      const int32_t *__restrict__ st_offs,
                                                      const uint8_t *__restrict__ st_mask,
                                                      const double *__restrict__ st_val,
                                                      const double *__restrict__ r_old, double *__restrict__ r_new,
                                                      const double *__restrict__ q, double *__restrict__ t,
                                                      double *__restrict__ out, Partials pq_in,
                                                      DevState *__restrict__ st, int32_t k) {
    __shared__ double sh[kWavesPerBlock];
    __shared__ double bc;
    if (st->done) return;
    const double pq = reduce_partials(pq_in, sh, &bc);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (is_block0_thread0()) {
            st->pq = pq;
            st->iter = k;
            st->done = kDoneBreakdown;
        }
        return;
    }
    const double alpha = st->rho[k & 1] / pq;
    if (is_block0_thread0()) {
        st->pq = pq;
        st->r_iter = k + 1;
    }
    const int lane = threadIdx.x & (kWave - 1);
    double acc = 0.0;
    TileWalk walk((m + kWave - 1) / kWave);
    for (int tl = walk.next(); tl >= 0; tl = walk.next()) {
        const int r0 = __builtin_amdgcn_readfirstlane(tl * kWave);
        const int nrows = min(kWave, m - r0);
        const int row = r0 + min(lane, nrows - 1);
        const int off = st_off[tl];
        const int width = (st_off[tl + 1] - off) / kWave;
        const uint32_t mask = st_mask[(int64_t)tl * kWave + lane];
        const double rv = fma(-alpha, q[row], r_old[row]);
        double w[kSliceMaxWidth], rn[kSliceMaxWidth];
#pragma unroll
        for (int j = 0; j < kSliceMaxWidth; ++j) {
            w[j] = rn[j] = 0.0;
            if (j < width) {   // uniform across the wavefront
                const int c = (mask >> j) & 1u ? row + st_offs[tl * kSliceMaxWidth + j] : row;
                w[j] = st_val[off + j * kWave + lane];
                rn[j] = fma(-alpha, q[c], r_old[c]);
            }
        }
        double s = 0.0;
        {
#pragma clang fp contract(off)
#pragma unroll
            for (int j = 0; j < kSliceMaxWidth; ++j)
                if ((mask >> j) & 1u) s = s + w[j] * rn[j];
        }
        if (lane < nrows) {
            r_new[row] = rv;
            t[row] = s;
            acc = fma(rv, rv, acc);
        }
    }
    const double sum = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = sum;
}

// x += alpha p, r -= alpha q; partial r^T r per workgroup.
__global__ __launch_bounds__(kBlock) void k_update_xr(int32_t m, double *__restrict__ x,
                                                      double *__restrict__ r,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ q,
                                                      double *__restrict__ out, Partials pq_in,
                                                      DevState *__restrict__ st, int device_coef,
                                                      int32_t k, double alpha_arg) {
    __shared__ double sh[kWavesPerBlock];
    __shared__ double bc;
    double alpha = alpha_arg;
    if (device_coef) {
        if (st->done) return;
        const double pq = reduce_partials(pq_in, sh, &bc);
        if (!(pq > 0.0) || !isfinite(pq)) {
            if (is_block0_thread0()) {
                st->pq = pq;
                st->iter = k;
                st->done = kDoneBreakdown;
            }
            return;
        }
        alpha = st->rho[k & 1] / pq;
        if (is_block0_thread0()) {
            st->pq = pq;
            st->r_iter = k + 1;
        }
    }
    double acc = 0.0;
    const int64_t npair = m >> 1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double2 *x2 = reinterpret_cast<double2 *>(x);
    double2 *r2 = reinterpret_cast<double2 *>(r);
    const double2 *p2 = reinterpret_cast<const double2 *>(p);
    const double2 *q2 = reinterpret_cast<const double2 *>(q);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npair; i += stride) {
        const double2 pv = p2[i], qv = q2[i];
        double2 xv = x2[i], rv = r2[i];
        xv.x = fma(alpha, pv.x, xv.x);
        xv.y = fma(alpha, pv.y, xv.y);
        rv.x = fma(-alpha, qv.x, rv.x);
        rv.y = fma(-alpha, qv.y, rv.y);
        x2[i] = xv;
        r2[i] = rv;
        acc = fma(rv.x, rv.x, acc);
        acc = fma(rv.y, rv.y, acc);
    }
    if ((m & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const int32_t i = m - 1;
        x[i] = fma(alpha, p[i], x[i]);
        const double rv = fma(-alpha, q[i], r[i]);
        r[i] = rv;
        acc = fma(rv, rv, acc);
    }
    const double s = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// p = r + beta p with beta from the host (split mode).
__global__ __launch_bounds__(kBlock) void k_update_p(int32_t m, const double *__restrict__ r,
                                                     double *__restrict__ p, double beta) {
    const int64_t npair = m >> 1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double2 *p2 = reinterpret_cast<double2 *>(p);
    const double2 *r2 = reinterpret_cast<const double2 *>(r);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npair; i += stride) {
        const double2 rv = r2[i];
        double2 pv = p2[i];
        pv.x = fma(beta, pv.x, rv.x);
        pv.y = fma(beta, pv.y, rv.y);
        p2[i] = pv;
    }
    if ((m & 1) && blockIdx.x == 0 && threadIdx.x == 0) p[m - 1] = fma(beta, p[m - 1], r[m - 1]);
}

// Float64 CG with device coefficients, x update deferred by one kernel.
// Algorithm 1 adds alpha p to x and subtracts alpha q from r in one step;
// x is not read again before the p update, which reads the same p, so the
// x update moves there: k_update_r forms r -= alpha q (partial r^T r per
// workgroup, p^T q recorded for the next kernel), and k_update_px forms
// x += alpha p with alpha recomputed from the same operands (bitwise the
// same value), then p = r + beta p unless the solve stops.  The x/r kernel
// no longer reads p: one pass over p per iteration less.
// On a breakdown only workgroup 0 acts (it records the state); a workgroup
// that starts after that store sees `done` and returns, so no work that
// every workgroup must do may hang on this branch.  The x term owed by the
// two-iteration update is added by k_update_pxb, which reads the recorded
// state after this kernel has completed.
__global__ __launch_bounds__(kBlock) void k_update_r(int32_t m, double *__restrict__ r,
                                                     const double *__restrict__ q,
                                                     double *__restrict__ out, Partials pq_in,
                                                     DevState *__restrict__ st, int32_t k) {
    __shared__ double sh[kWavesPerBlock];
    __shared__ double bc;
    if (st->done) return;
    const double pq = reduce_partials(pq_in, sh, &bc);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (is_block0_thread0()) {
            st->pq = pq;
            st->iter = k;
            st->done = kDoneBreakdown;
        }
        return;
    }
    const double alpha = st->rho[k & 1] / pq;
    if (is_block0_thread0()) {
        st->pq = pq;
        st->r_iter = k + 1;
    }
    double acc = 0.0;
    const int64_t npair = m >> 1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double2 *r2 = reinterpret_cast<double2 *>(r);
    const double2 *q2 = reinterpret_cast<const double2 *>(q);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npair; i += stride) {
        double2 rv = r2[i];
        const double2 qv = q2[i];
        rv.x = fma(-alpha, qv.x, rv.x);
        rv.y = fma(-alpha, qv.y, rv.y);
        r2[i] = rv;
        acc = fma(rv.x, rv.x, acc);
        acc = fma(rv.y, rv.y, acc);
    }
    if ((m & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const double rv = fma(-alpha, q[m - 1], r[m - 1]);
        r[m - 1] = rv;
        acc = fma(rv, rv, acc);
    }
    const double s = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_update_px(int32_t m, double *__restrict__ x,
                                                      const double *__restrict__ r,
                                                      double *__restrict__ p, Partials rr_in,
                                                      DevState *__restrict__ st, int32_t k) {
    __shared__ double sh[kWavesPerBlock];
    __shared__ double bc;
    // r of this iteration not updated (breakdown in k_update_r, or the solve
    // stopped earlier): x stays as it was.  `done` is not read here: workgroup
    // 0 of this kernel may set it before other workgroups start.
    if (st->r_iter != k + 1) return;
    const double rr = reduce_partials(rr_in, sh, &bc);
    const double rho_k = st->rho[k & 1];
    const double alpha = rho_k / st->pq;
    const double beta = rr / rho_k;
    const bool conv = stop_test(rr, st->bb, st->tol);
    const bool maxed = k + 1 >= st->maxit;
    const bool stop = conv || maxed;
    if (is_block0_thread0()) {
        st->rho[(k + 1) & 1] = rr;
        st->rr = rr;
        st->iter = k + 1;
        if (conv) st->done = kDoneConverged;
        else if (maxed) st->done = kDoneMaxit;
    }
    const int64_t npair = m >> 1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double2 *x2 = reinterpret_cast<double2 *>(x);
    double2 *p2 = reinterpret_cast<double2 *>(p);
    const double2 *r2 = reinterpret_cast<const double2 *>(r);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npair; i += stride) {
        double2 pv = p2[i];
        double2 xv = x2[i];
        xv.x = fma(alpha, pv.x, xv.x);
        xv.y = fma(alpha, pv.y, xv.y);
        x2[i] = xv;
        if (!stop) {
            const double2 rv = r2[i];
            pv.x = fma(beta, pv.x, rv.x);
            pv.y = fma(beta, pv.y, rv.y);
            p2[i] = pv;
        }
    }
    if ((m & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const double pv = p[m - 1];
        x[m - 1] = fma(alpha, pv, x[m - 1]);
        if (!stop) p[m - 1] = fma(beta, pv, r[m - 1]);
    }
}

// The end of plain CG's iteration k with x updated every other iteration
// (two p buffers): r^T r of the new residual from the r update's partials,
// beta, the stop test; workgroup 0 records iteration k+1 (and alpha_k at an
// even k that goes on).  Shared by k_update_pxb and k_spmv_dir.
struct CgCoef {
    double alpha, beta, alpha_prev;
    bool stop, odd;
};

__device__ __forceinline__ CgCoef cg_coef(const Partials &rr_in, DevState *st, int32_t k, double *sh,
                                          double *bc) {
    CgCoef c;
    const double rr = reduce_partials(rr_in, sh, bc);
    const double rho_k = st->rho[k & 1];
    c.alpha = rho_k / st->pq;
    c.beta = rr / rho_k;
    c.alpha_prev = st->alpha_prev;   // written at k - 1 (used at an odd k only)
    const bool conv = stop_test(rr, st->bb, st->tol);
    const bool maxed = k + 1 >= st->maxit;
    c.stop = conv || maxed;
    c.odd = k & 1;
    if (is_block0_thread0()) {
        st->rho[(k + 1) & 1] = rr;
        st->rr = rr;
        st->iter = k + 1;
        if (conv) st->done = kDoneConverged;
        else if (maxed) st->done = kDoneMaxit;
        if (!c.odd && !c.stop) st->alpha_prev = c.alpha;
    }
    return c;
}

// r of iteration k not updated (see k_update_px): after a breakdown in that
// r update at an odd k, x still owes alpha_{k-1} p_{k-1} (in p_oth).  Both
// fields were written by the previous kernel, so every workgroup reads the
// same values.
__device__ __forceinline__ void cg_breakdown_flush(int32_t m, double *x, const double *p_oth,
                                                   const DevState *st, int32_t k) {
    if ((k & 1) && st->done == kDoneBreakdown && st->iter == k) {
        const double ap = st->alpha_prev;
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock)
            x[i] = fma(ap, p_oth[i], x[i]);
    }
}

// k_update_px with x updated every other iteration (two p buffers, see the
// launcher's declaration): at an odd k the two owed terms are added with
// the same two fmas, in the same order, as by k_update_px at k-1 and k.
__global__ __launch_bounds__(kBlock) void k_update_pxb(int32_t m, double *__restrict__ x,
                                                       const double *__restrict__ r,
                                                       const double *__restrict__ p_cur,
                                                       double *__restrict__ p_oth, Partials rr_in,
                                                       DevState *__restrict__ st, int32_t k) {
    __shared__ double sh[kWavesPerBlock];
    __shared__ double bc;
    if (st->r_iter != k + 1) {
        cg_breakdown_flush(m, x, p_oth, st, k);
        return;
    }
    const CgCoef c = cg_coef(rr_in, st, k, sh, &bc);
    const double alpha = c.alpha, beta = c.beta, alpha_prev = c.alpha_prev;
    const bool stop = c.stop, odd = c.odd;
    const int64_t npair = m >> 1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double2 *x2 = reinterpret_cast<double2 *>(x);
    const double2 *pc2 = reinterpret_cast<const double2 *>(p_cur);
    double2 *po2 = reinterpret_cast<double2 *>(p_oth);
    const double2 *r2 = reinterpret_cast<const double2 *>(r);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npair; i += stride) {
        const double2 pc = pc2[i];
        if (odd) {
            const double2 po = po2[i];
            double2 xv = x2[i];
            xv.x = fma(alpha, pc.x, fma(alpha_prev, po.x, xv.x));
            xv.y = fma(alpha, pc.y, fma(alpha_prev, po.y, xv.y));
            x2[i] = xv;
        } else if (stop) {
            double2 xv = x2[i];
            xv.x = fma(alpha, pc.x, xv.x);
            xv.y = fma(alpha, pc.y, xv.y);
            x2[i] = xv;
        }
        if (!stop) {
            const double2 rv = r2[i];
            double2 pn;
            pn.x = fma(beta, pc.x, rv.x);
            pn.y = fma(beta, pc.y, rv.y);
            po2[i] = pn;
        }
    }
    if ((m & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const int32_t i = m - 1;
        const double pc = p_cur[i];
        if (odd) x[i] = fma(alpha, pc, fma(alpha_prev, p_oth[i], x[i]));
        else if (stop) x[i] = fma(alpha, pc, x[i]);
        if (!stop) p_oth[i] = fma(beta, pc, r[i]);
    }
}

// The end of preconditioned CG's iteration k from r^T r and r^T z of the new
// residual: alpha_k, beta, a breakdown (r^T z <= 0 or not finite while
// r != 0) and the stop test; workgroup 0 records iteration k+1.  Returns
// whether the solve stops.  Shared by k_update_p_pcg and k_spmv_dir.
__device__ __forceinline__ bool pcg_coef(double rr, double rz, DevState *st, int32_t k, double &alpha,
                                         double &beta) {
    const bool broke = (!(rz > 0.0) || !isfinite(rz)) && rr != 0.0;
    const bool conv = stop_test(rr, st->bb, st->tol);
    const bool maxed = k + 1 >= st->maxit;
    const double rho_k = st->rho[k & 1];
    beta = rz / rho_k;
    alpha = rho_k / st->pq;
    if (is_block0_thread0()) {
        st->rho[(k + 1) & 1] = rz;
        st->rr = rr;
        st->iter = k + 1;
        if (broke) st->done = kDoneBreakdown;
        else if (conv) st->done = kDoneConverged;
        else if (maxed) st->done = kDoneMaxit;
    }
    return broke || conv || maxed;
}

// Preconditioned CG: p = z + beta p with rho = r^T z (z = M^-1 r); the stop
// test is on r^T r.  first: setup step (after r = b - A x and z = M^-1 r):
// rho_0 = r^T z, ||b||^2 from bb_in, the stop test at the top of iteration 0,
// and p = z.  Otherwise after the r update of iteration k: x += alpha p when
// x is given (alpha = rho_k / p^T q as the r update formed it), then a
// breakdown (r^T z <= 0 or not finite while r != 0) ends the solve before
// the stop test; workgroup 0 records iteration k+1.  b = 0 stops at once
// (x = 0).
__global__ __launch_bounds__(kBlock) void k_update_p_pcg(int32_t m, const double *__restrict__ z,
                                                         double *__restrict__ p, double *__restrict__ x,
                                                         Partials rr_in, Partials rz_in, Partials bb_in,
                                                         DevState *__restrict__ st, int first,
                                                         int32_t k) {
    __shared__ double sh[2 * kWavesPerBlock];
    __shared__ double bc[2];
    // after iteration k: only if its r was updated (see k_update_px for why
    // `done` is not read)
    if (first ? st->done != 0 : st->r_iter != k + 1) return;
    double rr, rz;
    reduce_partials2(rr_in, rz_in, sh, bc, rr, rz);
    double beta = 0.0, alpha = 0.0;
    bool stop = false;
    if (first) {
        const double bb = reduce_partials(bb_in, sh, bc);
        const bool conv = stop_test(rr, bb, st->tol) || bb == 0.0;
        const bool stop0 = conv || st->maxit <= 0;
        if (is_block0_thread0()) {
            st->rho[0] = rz;
            st->rr = rr;
            st->bb = bb;
            st->iter = 0;
            if (stop0) st->done = conv ? kDoneConverged : kDoneMaxit;
        }
        if (stop0) return;
    } else {
        stop = pcg_coef(rr, rz, st, k, alpha, beta);
    }
    const bool upd_x = x && !first;
    if (stop && !upd_x) return;
    const int64_t npair = m >> 1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double2 *p2 = reinterpret_cast<double2 *>(p);
    double2 *x2 = reinterpret_cast<double2 *>(x);
    const double2 *z2 = reinterpret_cast<const double2 *>(z);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npair; i += stride) {
        double2 pv = p2[i];
        if (upd_x) {
            double2 xv = x2[i];
            xv.x = fma(alpha, pv.x, xv.x);
            xv.y = fma(alpha, pv.y, xv.y);
            x2[i] = xv;
        }
        if (!stop) {
            const double2 zv = z2[i];
            pv.x = fma(beta, pv.x, zv.x);
            pv.y = fma(beta, pv.y, zv.y);
            p2[i] = pv;
        }
    }
    if ((m & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const double pv = p[m - 1];
        if (upd_x) x[m - 1] = fma(alpha, pv, x[m - 1]);
        if (!stop) p[m - 1] = fma(beta, pv, z[m - 1]);
    }
}

// ---------------------------------------------------------------------------
// Direction update fused into the next SpMV (stencil slices, two rows per
// lane; plain CG with two p buffers, or preconditioned CG with its x update
// deferred).  One launch ends iteration k as k_update_pxb (PCG:
// k_update_p_pcg) does, with the same coefficient step, and runs the SpMV of
// iteration k+1 on p_{k+1} = d + beta p_k formed for every gathered column:
// q = A p_{k+1}, p_{k+1} written to the other p buffer for the lane's own
// rows, the owed x update there, and one p^T q partial per workgroup.  When
// iteration k ends the solve, the launch only completes x, as the separate
// kernel's stop path does, and records no partial.  x, p, q and the
// partials are bitwise those of the separate kernels on the same grid.
// Workgroup 0 records iteration k+1 in spmv_iter when its SpMV runs.
template <bool NT, bool PCG>
__global__ __launch_bounds__(kBlock) void k_spmv_dir(int32_t m, const int32_t *__restrict__ st_off,
                                                     const int32_t *__restrict__ st_offs,
                                                     const uint8_t *__restrict__ st_mask,
                                                     const double *__restrict__ st_val,
                                                     const double *__restrict__ p_cur,
                                                     const double *__restrict__ d, double *p_oth,
                                                     double *__restrict__ x, double *__restrict__ q,
                                                     double *__restrict__ out, Partials rr_in, Partials rz_in,
                                                     DevState *__restrict__ st, int32_t k) {
    __shared__ double sh[2 * kWavesPerBlock];
    __shared__ double bc[2];
    if (st->r_iter != k + 1) {
        if constexpr (!PCG) cg_breakdown_flush(m, x, p_oth, st, k);
        return;
    }
    DirArgs D{d, p_oth, x, 0.0, 0.0, 0.0, 0};
    bool stop;
    if constexpr (PCG) {
        double rr, rz;
        reduce_partials2(rr_in, rz_in, sh, bc, rr, rz);
        stop = pcg_coef(rr, rz, st, k, D.alpha, D.beta);
        D.xmode = 1;
    } else {
        const CgCoef c = cg_coef(rr_in, st, k, sh, bc);
        D.alpha = c.alpha;
        D.beta = c.beta;
        D.alpha_prev = c.alpha_prev;
        stop = c.stop;
        D.xmode = c.odd ? 2 : (stop ? 1 : 0);
    }
    if (stop) {
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock)
            x[i] = x_owed(D.xmode, x[i], D.alpha, p_cur[i], D.alpha_prev, D.xmode == 2 ? p_oth[i] : 0.0);
        return;
    }
    if (is_block0_thread0()) st->spmv_iter = k + 1;
    CsrDev A{};
    A.m = m;
    A.st_off = st_off;
    A.st_offs = st_offs;
    A.st_mask = st_mask;
    A.st_val = st_val;
    const SpmvArgs<double> a{p_cur, q, nullptr, nullptr, nullptr};
    double acc0 = 0.0;
    TileWalk walk(((m + kWave - 1) / kWave + 1) / 2);   // slice pairs
    spmv_sten2_wave<kSpmvDir, NT>(A, walk, a, acc0, D);
    const double s0 = block_sum<kBlock>(acc0, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s0;
}

// ---------------------------------------------------------------------------
// Mixed precision: float32 r, p, q with float64 x and float64 sums.

// x += alpha p (float64), r -= (float)alpha q (float32); partial r^T r in float64.
__global__ __launch_bounds__(kBlock) void k_update_xr_mixed(int32_t m, double *__restrict__ x,
                                                            float *__restrict__ r,
                                                            const float *__restrict__ p,
                                                            const float *__restrict__ q,
                                                            double *__restrict__ out,
                                                            Partials pq_in,
                                                            DevState *__restrict__ st, int32_t k) {
    __shared__ double sh[kWavesPerBlock];
    __shared__ double bc;
    if (st->done) return;
    const double pq = reduce_partials(pq_in, sh, &bc);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (is_block0_thread0()) {
            st->pq = pq;
            st->iter = k;
            st->done = kDoneBreakdown;
        }
        return;
    }
    const double alpha = st->rho[k & 1] / pq;
    const float alpha32 = (float)alpha;
    if (is_block0_thread0()) st->pq = pq;
    double acc = 0.0;
    const int64_t npair = m >> 1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double2 *x2 = reinterpret_cast<double2 *>(x);
    float2 *r2 = reinterpret_cast<float2 *>(r);
    const float2 *p2 = reinterpret_cast<const float2 *>(p);
    const float2 *q2 = reinterpret_cast<const float2 *>(q);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npair; i += stride) {
        const float2 pv = p2[i], qv = q2[i];
        double2 xv = x2[i];
        float2 rv = r2[i];
        xv.x = fma(alpha, (double)pv.x, xv.x);
        xv.y = fma(alpha, (double)pv.y, xv.y);
        rv.x = fmaf(-alpha32, qv.x, rv.x);
        rv.y = fmaf(-alpha32, qv.y, rv.y);
        x2[i] = xv;
        r2[i] = rv;
        acc = fma((double)rv.x, (double)rv.x, acc);
        acc = fma((double)rv.y, (double)rv.y, acc);
    }
    if ((m & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const int32_t i = m - 1;
        x[i] = fma(alpha, (double)p[i], x[i]);
        const float rv = fmaf(-alpha32, q[i], r[i]);
        r[i] = rv;
        acc = fma((double)rv, (double)rv, acc);
    }
    const double s = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// p = r + (float)beta p, or a refinement request when the float32 residual has
// dropped by delta since the last refinement or meets the tolerance.
__global__ __launch_bounds__(kBlock) void k_update_p_mixed(int32_t m, const float *__restrict__ r,
                                                           float *__restrict__ p, Partials rr_in,
                                                           DevState *__restrict__ st,
                                                           int device_coef, int32_t k,
                                                           double beta_arg) {
    __shared__ double sh[kWavesPerBlock];
    __shared__ double bc;
    double beta = beta_arg;
    if (device_coef) {
        if (st->done) return;
        const double rr = reduce_partials(rr_in, sh, &bc);
        const double rho_k = st->rho[k & 1];
        const bool refine = sqrt(rr) < st->delta * st->rmax || sqrt(rr) < st->tol * sqrt(st->bb);
        const bool maxed = k + 1 >= st->maxit;
        if (is_block0_thread0()) {
            st->rho[(k + 1) & 1] = rr;
            st->rr = rr;
            st->iter = k + 1;
            if (refine) st->done = kDoneRefine;
            else if (maxed) st->done = kDoneMaxit;
        }
        if (refine || maxed) return;
        beta = rr / rho_k;
    }
    const float beta32 = (float)beta;
    const int64_t npair = m >> 1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    float2 *p2 = reinterpret_cast<float2 *>(p);
    const float2 *r2 = reinterpret_cast<const float2 *>(r);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npair; i += stride) {
        const float2 rv = r2[i];
        float2 pv = p2[i];
        pv.x = fmaf(beta32, pv.x, rv.x);
        pv.y = fmaf(beta32, pv.y, rv.y);
        p2[i] = pv;
    }
    if ((m & 1) && blockIdx.x == 0 && threadIdx.x == 0) p[m - 1] = fmaf(beta32, p[m - 1], r[m - 1]);
}

// r32 = (float) r64 (and p32 = r32 with init_p); partial r32^T r32 in float64.
__global__ __launch_bounds__(kBlock) void k_convert_residual(int32_t m, const double *__restrict__ r64,
                                                             float *__restrict__ r32,
                                                             float *__restrict__ p32,
                                                             double *__restrict__ out, int init_p) {
    __shared__ double sh[kWavesPerBlock];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        const float v = (float)r64[i];
        r32[i] = v;
        if (init_p) p32[i] = v;
        acc = fma((double)v, (double)v, acc);
    }
    const double s = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void k_gather(int32_t cnt, const int32_t *__restrict__ idx, const double *__restrict__ src,
                         double *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) dst[i] = src[idx[i]];
}

__global__ void k_scatter(int32_t cnt, const int32_t *__restrict__ idx, const double *__restrict__ src,
                          double *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) dst[idx[i]] = src[i];
}

template <int MODE, class T>
void launch_spmv_mode(const CsrDev &A, const Schedule &S, int grid, const SpmvArgs<T> &a,
                      double *out, Partials in0, Partials in1, DevState *st, int flags,
                      hipStream_t s) {
    // stencil slices with two rows per lane where the 16-byte accesses are aligned
    const bool wide = sizeof(T) == 8 && (MODE == kSpmvPlain || MODE == kSpmvDot) &&
                      ((uintptr_t)a.q & 15) == 0 && (MODE != kSpmvDot || ((uintptr_t)a.p_own & 15) == 0);
    const int L = S.kind == kTileStencil ? (wide ? (S.stream_nt ? -9 : -8) : (S.stream_nt ? -7 : -6))
                  : S.kind == kTileSlicedDict ? (S.stream_nt ? -5 : -4)
                  : S.kind == kTileSliced ? (S.bins[0].lanes <= kSliceMaxWidth
                                                 ? (wide && A.sell_len
                                                        ? (A.sell_gap ? (S.stream_nt ? -13 : -12)
                                                                      : (S.stream_nt ? -11 : -10))
                                                        : (A.sell_gap ? -14 : -2))
                                                 : -3)
                  : S.kind == kTileStream ? -1
                  : (S.identity && S.nbins == 1 && S.huge_count == 0) ? S.bins[0].lanes : 0;
    const T *val, *sval;
    if constexpr (sizeof(T) == 8) {
        val = reinterpret_cast<const T *>(A.val);
        sval = reinterpret_cast<const T *>(A.sell_val);
    } else {
        val = reinterpret_cast<const T *>(A.val32);
        sval = reinterpret_cast<const T *>(A.sell_val32);
    }
#define CGMI_SPMV(FL)                                                                             \
    hipLaunchKernelGGL((k_spmv<MODE, FL, T>), dim3(grid), dim3(kBlock), 0, s, A.m, A.rp, A.ci, val, \
                       A.rows, A.sell_off, A.sell_ci, sval, A.sell_idx, A.sell_dict, A.col_base,       \
                       A.st_off, A.st_offs, A.st_mask, A.st_val, A.sell_len, A.tile_row, A.sell_lenx,   \
                       A.sell_gap, S, a, out, in0, in1, st, flags)
    switch (L) {
        case 1: CGMI_SPMV(1); break;
        case 2: CGMI_SPMV(2); break;
        case 4: CGMI_SPMV(4); break;
        case 8: CGMI_SPMV(8); break;
        case 16: CGMI_SPMV(16); break;
        case 32: CGMI_SPMV(32); break;
        case 64: CGMI_SPMV(64); break;
        case -1: CGMI_SPMV(-1); break;
        case -2: CGMI_SPMV(-2); break;
        case -3: CGMI_SPMV(-3); break;
        case -4: CGMI_SPMV(-4); break;
        case -5: CGMI_SPMV(-5); break;
        case -6: CGMI_SPMV(-6); break;
        case -7: CGMI_SPMV(-7); break;
        case -8: CGMI_SPMV(-8); break;
        case -9: CGMI_SPMV(-9); break;
        case -10: CGMI_SPMV(-10); break;
        case -11: CGMI_SPMV(-11); break;
        case -12: CGMI_SPMV(-12); break;
        case -13: CGMI_SPMV(-13); break;
        case -14: CGMI_SPMV(-14); break;
        default: CGMI_SPMV(0); break;
    }
#undef CGMI_SPMV
}

// q = A p as one accumulating pass per column block, between the start and
// finish kernels (same grid as the caller's partials).
template <class T>
void launch_spmv_blocked(const CsrDev &A, int grid, const SpmvArgs<T> &a, int mode, double *out,
                         Partials in0, Partials in1, DevState *st, int flags, hipStream_t s) {
    const ColBlocks &B = *A.cb;
    hipLaunchKernelGGL(k_blocked_start<T>, dim3(grid), dim3(kBlock), 0, s, A.m, a.q, in0, in1, st, flags);
    const int bflags = st ? kFlagCheckDone : 0;
    const Partials none{nullptr, 0};
    for (int b = 0; b < B.nb; ++b)
        launch_spmv_mode<kSpmvAccum, T>(B.dev[b], B.sched[b], B.grid[b], a, nullptr, none, none, st, bflags, s);
    if (mode == kSpmvDot)
        hipLaunchKernelGGL((k_blocked_finish<kSpmvDot, T>), dim3(grid), dim3(kBlock), 0, s, A.m, a, out, st, bflags);
    else if (mode == kSpmvResidual)
        hipLaunchKernelGGL((k_blocked_finish<kSpmvResidual, T>), dim3(grid), dim3(kBlock), 0, s, A.m, a, out, st,
                           bflags);
}

}  // namespace

hipError_t launch_spmv(const CsrDev &A, const Schedule &S, int grid, const double *p, double *q,
                       const double *p_own, const double *b, double *p_dst, double *out_partials,
                       Partials in0, Partials in1, DevState *st, int mode, int k0_check,
                       hipStream_t s) {
    if (A.m == 0) return hipSuccess;
    SpmvArgs<double> a{p, q, p_own, b, p_dst};
    if (S.kind == kTileColBlocked) {
        if (!A.cb || mode < kSpmvPlain || mode > kSpmvResidual) return hipErrorInvalidValue;
        const int flags = st ? (kFlagCheckDone | (mode == kSpmvDot && k0_check ? kFlagFirstIter : 0)) : 0;
        launch_spmv_blocked<double>(A, grid, a, mode, out_partials, in0, in1, st, flags, s);
        return hipGetLastError();
    }
    switch (mode) {
        case kSpmvPlain:
            launch_spmv_mode<kSpmvPlain, double>(A, S, grid, a, nullptr, in0, in1, st,
                                                 st ? kFlagCheckDone : 0, s);
            break;
        case kSpmvDot: {
            const int flags = st ? (kFlagCheckDone | (k0_check ? kFlagFirstIter : 0)) : 0;
            launch_spmv_mode<kSpmvDot, double>(A, S, grid, a, out_partials, in0, in1, st, flags, s);
            break;
        }
        case kSpmvResidual:
            launch_spmv_mode<kSpmvResidual, double>(A, S, grid, a, out_partials, in0, in1, nullptr, 0,
                                                    s);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_spmv_f32(const CsrDev &A, const Schedule &S, int grid, const float *p, float *q,
                           const float *p_own, double *out_partials, DevState *st, int mode,
                           hipStream_t s) {
    if (A.m == 0) return hipSuccess;
    if (S.kind == kTileStencil) return hipErrorInvalidValue;   // no float32 variant
    SpmvArgs<float> a{p, q, p_own, nullptr, nullptr};
    const Partials none{nullptr, 0};
    if (S.kind == kTileColBlocked) {
        if (!A.cb || (mode != kSpmvPlain && mode != kSpmvDot)) return hipErrorInvalidValue;
        launch_spmv_blocked<float>(A, grid, a, mode, out_partials, none, none, st, st ? kFlagCheckDone : 0, s);
        return hipGetLastError();
    }
    switch (mode) {
        case kSpmvPlain:
            launch_spmv_mode<kSpmvPlain, float>(A, S, grid, a, nullptr, none, none, nullptr, 0, s);
            break;
        case kSpmvDot:
            launch_spmv_mode<kSpmvDot, float>(A, S, grid, a, out_partials, none, none, st,
                                              st ? kFlagCheckDone : 0, s);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_update_xr(int32_t m, int grid, double *x, double *r, const double *p_own,
                            const double *q, double *out_partials, Partials pq, DevState *st,
                            int device_coef, int32_t k, double alpha_arg, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_xr, dim3(grid), dim3(kBlock), 0, s, m, x, r, p_own, q, out_partials,
                       pq, st, device_coef, k, alpha_arg);
    return hipGetLastError();
}

hipError_t launch_update_p(int32_t m, int grid, const double *r, double *p_own, double beta, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_p, dim3(grid), dim3(kBlock), 0, s, m, r, p_own, beta);
    return hipGetLastError();
}

hipError_t launch_pcg_xr_g(int32_t m, int grid, int width, const int32_t *grp, const int32_t *gci,
                           const double *gval, const double *r_old, double *r_new, const double *q,
                           double *t, double *out_partials, Partials pq, DevState *st, int32_t k,
                           hipStream_t s) {
    if (m == 0) return hipSuccess;
    if (width < 0 || width > kFusedGWidth) return hipErrorInvalidValue;
#define CGMI_PCG_XR_G(W)                                                                            \
    hipLaunchKernelGGL(k_pcg_xr_g<W>, dim3(grid), dim3(kBlock), 0, s, m, grp, gci, gval, r_old, r_new, q, t, \
                       out_partials, pq, st, k)
    if (width <= 1) CGMI_PCG_XR_G(1);
    else if (width <= 2) CGMI_PCG_XR_G(2);
    else if (width <= 4) CGMI_PCG_XR_G(4);
    else CGMI_PCG_XR_G(8);
#undef CGMI_PCG_XR_G
    return hipGetLastError();
}

hipError_t launch_pcg_xr_gs(int32_t m, int grid, const int32_t *st_off, const int32_t *st_offs,
                            const uint8_t *st_mask, const double *st_val, const double *r_old, double *r_new,
                            const double *q, double *t, double *out_partials, Partials pq, DevState *st,
                            int32_t k, hipStream_t s) {
    if (m == 0) return hipSuccess;
    if (grid < 8 || (grid & 7)) return hipErrorInvalidValue;   // the tile walk deals tiles out per XCD
    hipLaunchKernelGGL(k_pcg_xr_gs, dim3(grid), dim3(kBlock), 0, s, m, st_off, st_offs, st_mask, st_val, r_old,
                       r_new, q, t, out_partials, pq, st, k);
    return hipGetLastError();
}

hipError_t launch_update_r(int32_t m, int grid, double *r, const double *q, double *out, Partials pq,
                           DevState *st, int32_t k, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_r, dim3(grid), dim3(kBlock), 0, s, m, r, q, out, pq, st, k);
    return hipGetLastError();
}

hipError_t launch_update_pxb(int32_t m, int grid, double *x, const double *r, const double *p_cur,
                             double *p_oth, Partials rr, DevState *st, int32_t k, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_pxb, dim3(grid), dim3(kBlock), 0, s, m, x, r, p_cur, p_oth, rr, st, k);
    return hipGetLastError();
}

bool spmv_dir_applies(const CsrDev &A, const Schedule &S, int grid, const void *p_cur, const void *d,
                      const void *p_oth, const void *x, const void *q) {
    auto a16 = [](const void *v) { return ((uintptr_t)v & 15) == 0; };
    return S.kind == kTileStencil && A.st_val && A.col_base == 0 && A.m >= 2 && S.ntiles == (A.m + kWave - 1) / kWave &&
           grid >= 8 && (grid & 7) == 0 && a16(p_cur) && a16(d) && a16(p_oth) && a16(x) && a16(q);
}

hipError_t launch_spmv_dir(const CsrDev &A, const Schedule &S, int grid, const double *p_cur, const double *d,
                           double *p_oth, double *x, double *q, double *out, Partials rr, Partials rz,
                           DevState *st, int32_t k, int pcg, hipStream_t s) {
    if (A.m == 0) return hipSuccess;
    if (!spmv_dir_applies(A, S, grid, p_cur, d, p_oth, x, q) || !st || !out) return hipErrorInvalidValue;
#define CGMI_SPMV_DIR(NT, PCG)                                                                        \
    hipLaunchKernelGGL((k_spmv_dir<NT, PCG>), dim3(grid), dim3(kBlock), 0, s, A.m, A.st_off, A.st_offs,  \
                       A.st_mask, A.st_val, p_cur, d, p_oth, x, q, out, rr, rz, st, k)
    if (S.stream_nt) {
        if (pcg) CGMI_SPMV_DIR(true, true);
        else CGMI_SPMV_DIR(true, false);
    } else {
        if (pcg) CGMI_SPMV_DIR(false, true);
        else CGMI_SPMV_DIR(false, false);
    }
#undef CGMI_SPMV_DIR
    return hipGetLastError();
}

hipError_t launch_update_px(int32_t m, int grid, double *x, const double *r, double *p, Partials rr,
                            DevState *st, int32_t k, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_px, dim3(grid), dim3(kBlock), 0, s, m, x, r, p, rr, st, k);
    return hipGetLastError();
}

hipError_t launch_update_p_pcg(int32_t m, int grid, const double *z, double *p, double *x, Partials rr,
                               Partials rz, Partials bb, DevState *st, int first, int32_t k,
                               hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_p_pcg, dim3(grid), dim3(kBlock), 0, s, m, z, p, x, rr, rz, bb, st, first, k);
    return hipGetLastError();
}

hipError_t launch_gather(int32_t cnt, const int32_t *idx, const double *src, double *dst,
                         hipStream_t s) {
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3((cnt + 255) / 256), dim3(256), 0, s, cnt, idx, src, dst);
    return hipGetLastError();
}

hipError_t launch_scatter(int32_t cnt, const int32_t *idx, const double *src, double *dst,
                          hipStream_t s) {
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3((cnt + 255) / 256), dim3(256), 0, s, cnt, idx, src, dst);
    return hipGetLastError();
}

hipError_t launch_update_xr_mixed(int32_t m, int grid, double *x, float *r, const float *p,
                                  const float *q, double *out_partials, Partials pq, DevState *st,
                                  int32_t k, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_xr_mixed, dim3(grid), dim3(kBlock), 0, s, m, x, r, p, q,
                       out_partials, pq, st, k);
    return hipGetLastError();
}

hipError_t launch_update_p_mixed(int32_t m, int grid, const float *r, float *p, Partials rr,
                                 DevState *st, int device_coef, int32_t k, double beta_arg,
                                 hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_p_mixed, dim3(grid), dim3(kBlock), 0, s, m, r, p, rr, st,
                       device_coef, k, beta_arg);
    return hipGetLastError();
}

hipError_t launch_convert_residual(int32_t m, int grid, const double *r64, float *r32, float *p32,
                                   double *out_partials, int init_p, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_convert_residual, dim3(grid), dim3(kBlock), 0, s, m, r64, r32, p32,
                       out_partials, init_p);
    return hipGetLastError();
}

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
    return prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
}

}  // namespace cgmi
