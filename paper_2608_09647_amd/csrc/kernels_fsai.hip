// kernels_fsai.hip -- learned FSAI preconditioner kernels for gfx950.
//
// Network 12 -> 64 -> 64 -> 5 on the matrix cores, bfloat16 operands and
// float32 accumulation.  Activations are kept transposed (units x rows): the
// output fragment of a 16x16 product (lane l holds unit 4*(l/16)+v, row l%16)
// is a B-operand fragment of the next layer, so the forward pass needs no
// shuffles; weights are A-operand fragments held in registers.  A wavefront
// processes tiles of 16 rows.
//
// The contractions over 64 hidden units (layers 2 and 3 forward, W2^T in the
// backward pass) use the 16x16x32 form: its B operand (8 values per lane) is
// the concatenation of two 16-unit output fragments, i.e. lane l carries the
// units 32h + 16(j/4) + 4(l/16) + j%4, j = 0..7, and the weight fragments are
// loaded in that same unit order.  The contraction index is only summed over,
// so a common permutation of it in A and B leaves the product unchanged and
// costs no data movement.  Contractions of length 16 (12 features, 5
// outputs, and the weight gradients' sums over a tile's 16 rows) use the
// 16x16x16 form, which they fill exactly.
//
// The backward pass stages activations and signals in wavefront-private LDS in
// [unit][row] order so the weight-gradient products (a reduction over rows)
// read 4 consecutive rows per lane.
//
// Definitions (features, factor, loss) follow the header cgmi_fsai.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "cgmi_internal.h"
#include "fsai_internal.h"

namespace cgmi {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));   // bfloat16 bits
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kW = 64;

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// 16x16x16: lane l holds A[l%16][4(l/16)+v] and B[4(l/16)+v][l%16].
__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 16x16x32: eight contraction entries per lane, in the same positions for A
// and B.
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16v8, a),
                                                   __builtin_bit_cast(bf16v8, b), c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 cat(bf16x4 lo, bf16x4 hi) {
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Hidden unit carried by entry j of lane group q in contraction step h of a
// 16x16x32 product over 64 units.
__device__ __forceinline__ int unit32(int h, int q, int j) { return 32 * h + 16 * (j >> 2) + 4 * q + (j & 3); }

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// The parameters of one workgroup, rounded to bfloat16 once and staged in LDS
// zero-padded to 16-entry boundaries (features 12..15, outputs 5..15), so
// every fragment entry below is an unconditional LDS read.
struct ParamLds {
    uint16_t w1[kHidden][16];     // W1 [unit][feature]
    uint16_t w2[kHidden][kHidden];
    uint16_t w3[16][kHidden];     // W3 [output][unit]
    float b1[kHidden], b2[kHidden], b3[16];
};

// All threads of the workgroup take part; ends with a workgroup barrier.
__device__ __forceinline__ void stage_params(const float *__restrict__ th, ParamLds &P) {
    for (int i = threadIdx.x; i < kHidden * 16; i += blockDim.x) {
        const int u = i >> 4, k = i & 15;
        P.w1[u][k] = k < kFeat ? bf16_bits(th[kOffW1 + u * kFeat + k]) : 0;
        const int o = i >> 6, c = i & 63;
        P.w3[o][c] = o < kOut ? bf16_bits(th[kOffW3 + o * kHidden + c]) : 0;
    }
    for (int i = threadIdx.x; i < kHidden * kHidden; i += blockDim.x) P.w2[i >> 6][i & 63] = bf16_bits(th[kOffW2 + i]);
    for (int i = threadIdx.x; i < kHidden; i += blockDim.x) {
        P.b1[i] = th[kOffB1 + i];
        P.b2[i] = th[kOffB2 + i];
        if (i < 16) P.b3[i] = i < kOut ? th[kOffB3 + i] : 0.f;
    }
    __syncthreads();
}

__device__ __forceinline__ bf16x4 lds4(const uint16_t *p) {
    const uint2 u = *reinterpret_cast<const uint2 *>(p);
    bf16x4 b;
    b[0] = (short)(u.x & 0xFFFF);
    b[1] = (short)(u.x >> 16);
    b[2] = (short)(u.y & 0xFFFF);
    b[3] = (short)(u.y >> 16);
    return b;
}

// Weight fragments (A operands).
struct Frags {
    bf16x4 w1[4];      // W1: M-tile t (units 16t..), K = features (12 used of 16)
    bf16x8 w2[4][2];   // W2: M-tile t (out units), k-step h (in units unit32(h, ..))
    bf16x8 w3[2];      // W3: M = outputs (5 used of 16), k-step h
};

__device__ __forceinline__ void load_frags(const ParamLds &P, Frags &F) {
    const int l = threadIdx.x & (kW - 1);
    const int r = l & 15, q = l >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) F.w1[t] = lds4(&P.w1[16 * t + r][4 * q]);
    // unit32(h, q, 0..3) and unit32(h, q, 4..7) are runs of 4 consecutive units
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h)
            F.w2[t][h] = cat(lds4(&P.w2[16 * t + r][unit32(h, q, 0)]), lds4(&P.w2[16 * t + r][unit32(h, q, 4)]));
#pragma unroll
    for (int h = 0; h < 2; ++h) F.w3[h] = cat(lds4(&P.w3[r][unit32(h, q, 0)]), lds4(&P.w3[r][unit32(h, q, 4)]));
}

struct Fwd {
    f32x4 z1[4], z2[4];   // pre-activations (units 16t + 4q + v, row r)
    bf16x8 h1[2], h2[2];  // bfloat16 activations as 16x16x32 B fragments:
                          // entry 4(t%2)+v of h[t/2] is unit 16t + 4q + v
    f32x4 o;              // outputs 4q + v (valid < 5), row r
};

// Forward pass of one 16-row tile; fin: the lane's 4 feature bits (features
// 4q..4q+3 of row r).
__device__ __forceinline__ void forward_tile(const Frags &W, const ParamLds &P,
                                             bf16x4 fin, Fwd &Y) {
    const int l = threadIdx.x & (kW - 1);
    const int q = l >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        Y.z1[t] = mfma(W.w1[t], fin, zero4());
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            Y.z1[t][v] += P.b1[16 * t + 4 * q + v];
            Y.h1[t >> 1][4 * (t & 1) + v] = (short)bf16_bits(fmaxf(Y.z1[t][v], 0.f));
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 c = zero4();
#pragma unroll
        for (int h = 0; h < 2; ++h) c = mfma32(W.w2[t][h], Y.h1[h], c);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            c[v] += P.b2[16 * t + 4 * q + v];
            Y.h2[t >> 1][4 * (t & 1) + v] = (short)bf16_bits(fmaxf(c[v], 0.f));
        }
        Y.z2[t] = c;
    }
    f32x4 c = zero4();
#pragma unroll
    for (int h = 0; h < 2; ++h) c = mfma32(W.w3[h], Y.h2[h], c);
#pragma unroll
    for (int v = 0; v < 4; ++v) c[v] += P.b3[4 * q + v];
    Y.o = c;
}

__device__ __forceinline__ bf16x4 load_feats(const uint16_t *__restrict__ feats, int64_t row) {
    const int q = (threadIdx.x & (kW - 1)) >> 4;
    const uint2 u = *reinterpret_cast<const uint2 *>(feats + row * kFeatPad + 4 * q);
    bf16x4 b;
    b[0] = (short)(u.x & 0xFFFF);
    b[1] = (short)(u.x >> 16);
    b[2] = (short)(u.y & 0xFFFF);
    b[3] = (short)(u.y >> 16);
    return b;
}

// ---------------------------------------------------------------------------
// Stencil slots, scaled operator and features (thread per row).
__global__ void k_fsai_prepare(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               const double *__restrict__ val, int32_t *__restrict__ scol,
                               float *__restrict__ sval, double *__restrict__ diag,
                               uint16_t *__restrict__ feats, int32_t *__restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int col[kSlots];
    double a[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        col[s] = -1;
        a[s] = 0.0;
    }
    int bad = 0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int c = ci[k];
        const int s = stencil_slot(i, c);
        if (col[s] >= 0) bad = 1;
        col[s] = c;
        a[s] = val[k];
    }
    const double di = a[kSlotC];
    if (col[kSlotC] < 0 || !(di > 0.0)) bad = 1;
    if (bad) {
        atomicAdd(err, 1);
        return;
    }
    diag[i] = di;
    float f[kFeatPad];
#pragma unroll
    for (int k = 0; k < kFeatPad; ++k) f[k] = 0.f;
    scol[i * kSlots + kSlotC] = i;
    sval[i * kSlots + kSlotC] = 1.f;
    const int nb[4] = {kSlotW, kSlotE, kSlotS, kSlotN};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int s = nb[m];
        const int j = col[s];
        scol[i * kSlots + s] = j;
        if (j < 0) {
            sval[i * kSlots + s] = 0.f;
            f[8 + m] = 1.f;
            continue;
        }
        double dj = 0.0;
        for (int k = rp[j]; k < rp[j + 1]; ++k)
            if (ci[k] == j) dj = val[k];
        if (!(dj > 0.0)) {
            atomicAdd(err, 1);
            return;
        }
        const double ah = a[s] / sqrt(di * dj);
        sval[i * kSlots + s] = (float)ah;
        f[m] = (float)ah;
        f[4 + m] = (float)log(dj / di);
    }
#pragma unroll
    for (int k = 0; k < kFeatPad; ++k) feats[(int64_t)i * kFeatPad + k] = bf16_bits(f[k]);
}

// ---------------------------------------------------------------------------
// Forward pass over a list of 16-row tiles.  Training: outputs to out[row][8].
// Inference: the factor's values into G (CSR of tril(A)) and G^T.
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_fsai_forward(int32_t ntiles, const int32_t *__restrict__ tiles,
                                                      int64_t nrows, const uint16_t *__restrict__ feats,
                                                      const float *__restrict__ th, float *__restrict__ out,
                                                      const int32_t *__restrict__ scol,
                                                      const double *__restrict__ diag,
                                                      const int32_t *__restrict__ gpos,
                                                      const int32_t *__restrict__ tpos,
                                                      double *__restrict__ gval,
                                                      double *__restrict__ gtval,
                                                      int64_t *__restrict__ dg_zero) {
    __shared__ ParamLds P;
    stage_params(th, P);
    Frags W;
    load_frags(P, W);
    const int l = threadIdx.x & (kW - 1);
    const int r = l & 15, q = l >> 4;
    const int wave = blockIdx.x * (blockDim.x / kW) + threadIdx.x / kW;
    const int nwaves = gridDim.x * (blockDim.x / kW);
    for (int t = wave; t < ntiles; t += nwaves) {
        const int64_t row0 = tiles ? (int64_t)tiles[t] : (int64_t)t * 16;
        const int64_t row = row0 + r;
        const bf16x4 fin = row < nrows ? load_feats(feats, row) : bf16x4{0, 0, 0, 0};
        Fwd Y;
        forward_tile(W, P, fin, Y);
        if (row >= nrows) continue;
        if (TRAIN) {
            // outputs 0..7 of the row (5..7 are exact zeros: zero weights and
            // bias), and the row's dL/dG~ cleared for the loss to accumulate into
            if (q < kOutPad / 4)
                *reinterpret_cast<float4 *>(out + row * kOutPad + 4 * q) =
                    make_float4(Y.o[0], Y.o[1], Y.o[2], Y.o[3]);
            else if (q == 2)
                for (int b = 0; b < 3; ++b) dg_zero[row * 3 + b] = 0;
        } else if (q == 0) {
            // lanes 0..15 hold o_C, o_W, o_E, o_S of their row
            const double oc = Y.o[0], ow = Y.o[1], os = Y.o[3];
            const double sp = oc > 30.0 ? oc : log1p(exp(oc));
            const double gt[3] = {sp + kEpsDiag, ow, os};   // C, W, S
            const int slots[3] = {kSlotC, kSlotW, kSlotS};
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const int p = gpos[row * 3 + m];
                if (p < 0) continue;
                const int j = scol[row * kSlots + slots[m]];
                const double g = gt[m] / sqrt(diag[j]);
                gval[p] = g;
                gtval[tpos[p]] = g;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Loss and dL/dG~ on sampled rows, one wavefront per sample.  G~ of a row is
// read from the network outputs; A_hat from the slot tables.  dG~
// accumulates in 64-bit fixed point (each float term rounded to a multiple
// of 2^-40, then integer atomics): the sum does not depend on the order the
// atomics land in, so training is reproducible run to run.
constexpr double kDgScale = 1099511627776.0;   // 2^40

__device__ __forceinline__ void dg_add(int64_t *p, float x) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p),
              (unsigned long long)__double2ll_rn((double)x * kDgScale));
}
struct GRow {
    int col[3];      // C, W, S columns (-1 absent)
    float val[3];
};

__device__ __forceinline__ GRow g_row(int64_t base, int j, const float *__restrict__ out,
                                      const int32_t *__restrict__ scol) {
    GRow g;
    const float *o = out + (base + j) * kOutPad;
    const float oc = o[0];
    g.col[0] = j;
    g.val[0] = (oc > 30.f ? oc : log1pf(expf(oc))) + (float)kEpsDiag;
    g.col[1] = scol[(base + j) * kSlots + kSlotW];
    g.val[1] = g.col[1] >= 0 ? o[1] : 0.f;
    g.col[2] = scol[(base + j) * kSlots + kSlotS];
    g.val[2] = g.col[2] >= 0 ? o[3] : 0.f;
    return g;
}

__device__ __forceinline__ float ahat(int64_t base, int row, int colj, const int32_t *__restrict__ scol,
                                      const float *__restrict__ sval) {
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
        if (scol[(base + row) * kSlots + s] == colj) return sval[(base + row) * kSlots + s];
    return 0.f;
}

// Row i of G~ A_hat has at most 15 terms (G~ entry a of row i times slot s
// of row col_a(i)); lane t = 5a + s holds term t's column and value, and
// u_c is the sum, in term order, of the terms with column c.  The rows j
// with (G~ A_hat G~^T)_ij possibly nonzero are those whose pattern {j, W(j),
// S(j)} meets supp(u): for each term's column c, lane 3t + m proposes j =
// c, c + 1 (the row whose W slot is c) or the row whose S slot is c, and
// the lowest lane proposing a given j whose pattern holds c computes its
// entry e_ij = (G~ A_hat G~^T)_ij - delta_ij, adds e_ij^2 to the loss and
// its share of dL/dG~: coef e_ij u at j's columns into row j, and coef e_ij
// (G~ A_hat)_{j, col_b(i)} into row i (summed over the wave, one atomic
// per entry).
constexpr int kLossTerms = 3 * kSlots;

__global__ __launch_bounds__(256) void k_fsai_loss(int32_t nsamp, const int32_t *__restrict__ samp_row,
                                                   const int64_t *__restrict__ samp_base,
                                                   const int32_t *__restrict__ samp_n,
                                                   const float *__restrict__ out,
                                                   const int32_t *__restrict__ scol,
                                                   const float *__restrict__ sval,
                                                   int64_t *__restrict__ dg, float coef,
                                                   double *__restrict__ partials) {
    __shared__ double sh[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double loss = 0.0;
    for (int sidx = blockIdx.x * 4 + wv; sidx < nsamp; sidx += gridDim.x * 4) {
        const int i = samp_row[sidx];
        const int64_t base = samp_base[sidx];
        const int n = samp_n[sidx];
        const GRow gi = g_row(base, i, out, scol);
        // term t of u (lanes 0..14; -1: absent)
        int tcol = -1;
        float tval = 0.f;
        if (lane < kLossTerms) {
            const int a = lane / kSlots, sl = lane % kSlots;
            const int k = a == 0 ? gi.col[0] : a == 1 ? gi.col[1] : gi.col[2];
            const float ga = a == 0 ? gi.val[0] : a == 1 ? gi.val[1] : gi.val[2];
            if (k >= 0) {
                tcol = scol[(base + k) * kSlots + sl];
                if (tcol >= 0) tval = ga * sval[(base + k) * kSlots + sl];
            }
        }
        // candidate row of lane q = 3t + m
        const int t = min(lane / 3, kLossTerms - 1), m = lane % 3;
        const int c = __shfl(tcol, t, 64);
        int j = -1;
        if (lane < 3 * kLossTerms && c >= 0)
            j = m == 0 ? c : m == 1 ? c + 1 : scol[(base + c) * kSlots + kSlotN];
        GRow gj{{-1, -1, -1}, {0.f, 0.f, 0.f}};
        if (j >= 0 && j < n) {
            gj = g_row(base, j, out, scol);
            if (gj.col[0] != c && gj.col[1] != c && gj.col[2] != c) j = -1;
        } else {
            j = -1;
        }
        // the lowest lane proposing j owns it
        bool own = j >= 0;
        for (int q = 0; q < 3 * kLossTerms; ++q) {
            const int jq = __shfl(j, q, 64);
            if (q < lane && jq == j) own = false;
        }
        // u at j's columns (every lane takes part in the shuffles)
        float ub[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < kLossTerms; ++q) {
            const int cq = __shfl(tcol, q, 64);
            const float vq = __shfl(tval, q, 64);
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (cq >= 0 && cq == gj.col[b]) ub[b] += vq;
        }
        float gacc[3] = {0.f, 0.f, 0.f};
        if (own) {
            float mij = 0.f;
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (gj.col[b] >= 0) mij += gj.val[b] * ub[b];
            const float e = mij - (j == i ? 1.f : 0.f);
            loss += (double)e * (double)e;
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (gj.col[b] >= 0) dg_add(&dg[(base + j) * 3 + b], coef * e * ub[b]);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int cb = gi.col[b];
                if (cb < 0) continue;
                float w = 0.f;
#pragma unroll
                for (int s2 = 0; s2 < 3; ++s2) {
                    const int cs = gj.col[s2];
                    if (cs < 0) continue;
                    w += gj.val[s2] * ahat(base, cs, cb, scol, sval);
                }
                gacc[b] = coef * e * w;
            }
        }
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) gacc[b] += __shfl_xor(gacc[b], o, 64);
        if (lane == 0)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (gi.col[b] >= 0) dg_add(&dg[(base + i) * 3 + b], gacc[b]);
    }
    // per-block loss partial
    double v = loss;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// ---------------------------------------------------------------------------
// Backward pass over a list of 16-row tiles; one partial gradient per
// workgroup (waves added in order through LDS).
struct alignas(16) WaveLds {   // 8-byte loads of 4 consecutive entries
    uint16_t fT[16][16];    // [feature][row]
    uint16_t h1T[64][16];   // [unit][row]
    uint16_t h2T[64][16];
    uint16_t d1T[64][16];   // dz1
    uint16_t d2T[64][16];   // dz2
    uint16_t d3T[16][16];   // dz3 (outputs padded to 16)
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(256) void k_fsai_backward(int32_t ntiles, const int32_t *__restrict__ tiles,
                                                       const uint16_t *__restrict__ feats,
                                                       const float *__restrict__ th,
                                                       const float *__restrict__ out,
                                                       const int64_t *__restrict__ dg,
                                                       const int32_t *__restrict__ scol,
                                                       float *__restrict__ gpart) {
    __shared__ WaveLds L[4];
    __shared__ float acc[kNParams];
    const int l = threadIdx.x & (kW - 1);
    const int r = l & 15, q = l >> 4;
    const int wv = threadIdx.x / kW;
    WaveLds &S = L[wv];
    __shared__ ParamLds P;
    stage_params(th, P);
    Frags W;
    load_frags(P, W);
    // transposed weights for the backward products (A operands)
    bf16x4 w3t[4];     // W3^T: M-tile t (units), K = outputs (5 used of 16)
    bf16x8 w2t[4][2];  // W2^T: M-tile t (in units), k-step h (out units unit32(h, ..))
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) w3t[t][v] = (short)P.w3[4 * q + v][16 * t + r];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int j = 0; j < 8; ++j) w2t[t][h][j] = (short)P.w2[unit32(h, q, j)][16 * t + r];
    f32x4 gw1[4], gw2[4][4], gw3[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        gw1[t] = zero4();
        gw3[t] = zero4();
#pragma unroll
        for (int s = 0; s < 4; ++s) gw2[t][s] = zero4();
    }
    float gb1[4][4], gb2[4][4], gb3[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) gb1[t][v] = gb2[t][v] = 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) gb3[v] = 0.f;

    const int wave = blockIdx.x * 4 + wv;
    const int nwaves = gridDim.x * 4;
    for (int tt = wave; tt < ntiles; tt += nwaves) {
        const int64_t row = (int64_t)tiles[tt] + r;
        const bf16x4 fin = load_feats(feats, row);
        Fwd Y;
        forward_tile(W, P, fin, Y);
#pragma unroll
        for (int v = 0; v < 4; ++v) S.fT[4 * q + v][r] = (uint16_t)fin[v];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                S.h1T[16 * t + 4 * q + v][r] = (uint16_t)Y.h1[t >> 1][4 * (t & 1) + v];
                S.h2T[16 * t + 4 * q + v][r] = (uint16_t)Y.h2[t >> 1][4 * (t & 1) + v];
            }
        // dz3 (outputs 4q+v of row r)
        // dL/do of row r from dL/dG~: through the softplus for C, directly for
        // the W and S slots the row has, zero for the unused E and N
        bf16x4 d3;
        const float oc = out[row * kOutPad];
        const float sig = 1.f / (1.f + expf(-oc));
        float dgr[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) dgr[b] = (float)((double)dg[row * 3 + b] * (1.0 / kDgScale));
        const float dv[4] = {dgr[0] * sig, scol[row * kSlots + kSlotW] >= 0 ? dgr[1] : 0.f,
                             0.f, scol[row * kSlots + kSlotS] >= 0 ? dgr[2] : 0.f};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int o = 4 * q + v;
            const float g = q == 0 ? dv[v] : 0.f;
            gb3[v] += g;
            d3[v] = (short)bf16_bits(g);
            S.d3T[o][r] = (uint16_t)d3[v];
        }
        // dz2 = (W3^T dz3) * (z2 > 0)
        bf16x4 d2[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const f32x4 c = mfma(w3t[t], d3, zero4());
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float g = Y.z2[t][v] > 0.f ? c[v] : 0.f;
                gb2[t][v] += g;
                d2[t][v] = (short)bf16_bits(g);
                S.d2T[16 * t + 4 * q + v][r] = (uint16_t)d2[t][v];
            }
        }
        // dz1 = (W2^T dz2) * (z1 > 0)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 c = zero4();
#pragma unroll
            for (int h = 0; h < 2; ++h) c = mfma32(w2t[t][h], cat(d2[2 * h], d2[2 * h + 1]), c);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float g = Y.z1[t][v] > 0.f ? c[v] : 0.f;
                gb1[t][v] += g;
                S.d1T[16 * t + 4 * q + v][r] = bf16_bits(g);
            }
        }
        wave_sync();
        // weight gradients: sums over the tile's 16 rows
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bf16x4 a1 = lds4(&S.d1T[16 * t + r][4 * q]);
            gw1[t] = mfma(a1, lds4(&S.fT[r][4 * q]), gw1[t]);
            const bf16x4 a2 = lds4(&S.d2T[16 * t + r][4 * q]);
#pragma unroll
            for (int s = 0; s < 4; ++s) gw2[t][s] = mfma(a2, lds4(&S.h1T[16 * s + r][4 * q]), gw2[t][s]);
            gw3[t] = mfma(lds4(&S.d3T[r][4 * q]), lds4(&S.h2T[16 * t + r][4 * q]), gw3[t]);
        }
        wave_sync();
    }
    // bias sums: reduce over the 16 rows held by lanes r = 0..15
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int m = 1; m < 16; m <<= 1) {
                gb1[t][v] += __shfl_xor(gb1[t][v], m, 64);
                gb2[t][v] += __shfl_xor(gb2[t][v], m, 64);
            }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) gb3[v] += __shfl_xor(gb3[v], m, 64);
    // add the four wavefronts' gradients in order
    for (int p = threadIdx.x; p < kNParams; p += blockDim.x) acc[p] = 0.f;
    __syncthreads();
    for (int w = 0; w < 4; ++w) {
        if (wv == w) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int u = 16 * t + 4 * q + v;  // row of the gradient tile
                    if (r < kFeat) acc[kOffW1 + u * kFeat + r] += gw1[t][v];
#pragma unroll
                    for (int s = 0; s < 4; ++s) acc[kOffW2 + u * kHidden + 16 * s + r] += gw2[t][s][v];
                    const int o = 4 * q + v;
                    if (o < kOut) acc[kOffW3 + o * kHidden + 16 * t + r] += gw3[t][v];
                    if (r == 0) {
                        acc[kOffB1 + u] += gb1[t][v];
                        acc[kOffB2 + u] += gb2[t][v];
                    }
                }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = 4 * q + v;
                if (r == 0 && o < kOut) acc[kOffB3 + o] += gb3[v];
            }
        }
        __syncthreads();
    }
    for (int p = threadIdx.x; p < kNParams; p += blockDim.x)
        gpart[(int64_t)blockIdx.x * kNParams + p] = acc[p];
}

// Sum of the workgroup gradients in a fixed order; Adam step when t_step > 0,
// else the gradient is only written to grad_out.  A workgroup takes 64
// parameters; wave w sums, in order, the w-th quarter of the partials of
// its lane's parameter (16 loads in flight per lane), and wave 0 adds the
// four quarter sums in order.
__global__ __launch_bounds__(256) void k_fsai_adam(int32_t nparts, const float *__restrict__ gpart,
                                                   float *__restrict__ theta, float *__restrict__ m,
                                                   float *__restrict__ v, float *__restrict__ grad_out,
                                                   int32_t t_step, float lr) {
    __shared__ float part[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    const int pc = p < kNParams ? p : kNParams - 1;
    const int q = (nparts + 3) / 4;
    const int b0 = min(nparts, w * q), b1 = min(nparts, b0 + q);
    float g = 0.f;
    int b = b0;
    for (; b + 16 <= b1; b += 16) {
        float x[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) x[k] = gpart[(int64_t)(b + k) * kNParams + pc];
#pragma unroll
        for (int k = 0; k < 16; ++k) g += x[k];
    }
    for (; b < b1; ++b) g += gpart[(int64_t)b * kNParams + pc];
    part[w][lane] = g;
    __syncthreads();
    if (w != 0 || p >= kNParams) return;
    g = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    if (grad_out) grad_out[p] = g;
    if (t_step <= 0) return;
    const float be1 = 0.9f, be2 = 0.999f;
    const float mm = be1 * m[p] + (1.f - be1) * g;
    const float vv = be2 * v[p] + (1.f - be2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.f - powf(be1, (float)t_step));
    const float vh = vv / (1.f - powf(be2, (float)t_step));
    theta[p] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

// Thread per (slice, lane): copy the row's values into its slots.
__global__ void k_sell_refresh(int32_t m, int32_t ntiles, const int32_t *__restrict__ rp,
                               const int32_t *__restrict__ sell_off, const double *__restrict__ val,
                               double *__restrict__ sell_val) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t t = (int32_t)(g / 64), l = (int32_t)(g % 64);
    if (t >= ntiles) return;
    const int32_t i = t * 64 + l;
    if (i >= m) return;
    const int32_t b = rp[i], len = rp[i + 1] - rp[i];
    const int32_t w = (sell_off[t + 1] - sell_off[t]) / 64;
    for (int32_t j = 0; j < len && j < w; ++j) sell_val[(int64_t)sell_off[t] + (int64_t)j * 64 + l] = val[b + j];
}

// Thread per (slice, lane): scatter the row's values to the slots its mask
// marks, in order.
__global__ void k_stencil_refresh(int32_t m, int32_t ntiles, const int32_t *__restrict__ rp,
                                  const int32_t *__restrict__ st_off, const uint8_t *__restrict__ st_mask,
                                  const double *__restrict__ val, double *__restrict__ st_val) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t t = (int32_t)(g / 64), l = (int32_t)(g % 64);
    if (t >= ntiles) return;
    const int32_t i = t * 64 + l;
    if (i >= m) return;
    const int32_t b = rp[i], len = rp[i + 1] - rp[i];
    const int32_t w = (st_off[t + 1] - st_off[t]) / 64;
    uint32_t bits = st_mask[i];
    for (int32_t k = 0; k < len && bits; ++k) {
        const int32_t e = __builtin_ctz(bits);
        bits &= bits - 1;
        if (e < w) st_val[(int64_t)st_off[t] + (int64_t)e * 64 + l] = val[b + k];
    }
}

}  // namespace

// ---- launch wrappers -------------------------------------------------------

hipError_t fsai_prepare(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
                        int32_t *scol, float *sval, double *diag, uint16_t *feats, int32_t *err,
                        hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fsai_prepare, dim3((n + 255) / 256), dim3(256), 0, s, n, rp, ci, val, scol,
                       sval, diag, feats, err);
    return hipGetLastError();
}

hipError_t fsai_forward_outputs(int32_t ntiles, const int32_t *tiles, int64_t nrows,
                                const uint16_t *feats, const float *theta, float *out, int64_t *dg_zero,
                                hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    const int grid = (ntiles + 3) / 4 < 1024 ? (ntiles + 3) / 4 : 1024;
    hipLaunchKernelGGL(k_fsai_forward<true>, dim3(grid), dim3(256), 0, s, ntiles, tiles, nrows, feats,
                       theta, out, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, dg_zero);
    return hipGetLastError();
}

hipError_t fsai_forward_factor(int32_t n, const uint16_t *feats, const float *theta,
                               const int32_t *scol, const double *diag, const int32_t *gpos,
                               const int32_t *tpos, double *gval, double *gtval, hipStream_t s) {
    const int32_t ntiles = (n + 15) / 16;
    if (ntiles <= 0) return hipSuccess;
    const int grid = (ntiles + 3) / 4 < 2048 ? (ntiles + 3) / 4 : 2048;
    hipLaunchKernelGGL(k_fsai_forward<false>, dim3(grid), dim3(256), 0, s, ntiles, nullptr, (int64_t)n,
                       feats, theta, nullptr, scol, diag, gpos, tpos, gval, gtval, nullptr);
    return hipGetLastError();
}

hipError_t fsai_loss(int32_t nsamp, const int32_t *samp_row, const int64_t *samp_base,
                     const int32_t *samp_n, const float *out, const int32_t *scol, const float *sval,
                     int64_t *dg, float coef, double *partials, hipStream_t s) {
    if (nsamp <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fsai_loss, dim3(fsai_loss_blocks(nsamp)), dim3(256), 0, s, nsamp, samp_row,
                       samp_base, samp_n, out, scol, sval, dg, coef, partials);
    return hipGetLastError();
}

hipError_t fsai_backward(int32_t ntiles, const int32_t *tiles, const uint16_t *feats, const float *theta,
                         const float *out, const int64_t *dg, const int32_t *scol, float *gpart, int32_t grid,
                         hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fsai_backward, dim3(grid), dim3(256), 0, s, ntiles, tiles, feats, theta, out, dg,
                       scol, gpart);
    return hipGetLastError();
}

hipError_t fsai_adam(int32_t nparts, const float *gpart, float *theta, float *m, float *v,
                     float *grad_out, int32_t t_step, float lr, hipStream_t s) {
    hipLaunchKernelGGL(k_fsai_adam, dim3((kNParams + 63) / 64), dim3(256), 0, s, nparts, gpart, theta,
                       m, v, grad_out, t_step, lr);
    return hipGetLastError();
}

hipError_t sell_refresh(int32_t m, int32_t ntiles, const int32_t *rp, const int32_t *sell_off,
                        const double *val, double *sell_val, hipStream_t s) {
    if (m <= 0 || ntiles <= 0) return hipSuccess;
    const int64_t threads = (int64_t)ntiles * 64;
    hipLaunchKernelGGL(k_sell_refresh, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, m, ntiles,
                       rp, sell_off, val, sell_val);
    return hipGetLastError();
}

hipError_t stencil_refresh(int32_t m, int32_t ntiles, const int32_t *rp, const int32_t *st_off,
                           const uint8_t *st_mask, const double *val, double *st_val, hipStream_t s) {
    if (m <= 0 || ntiles <= 0) return hipSuccess;
    const int64_t threads = (int64_t)ntiles * 64;
    hipLaunchKernelGGL(k_stencil_refresh, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, m,
                       ntiles, rp, st_off, st_mask, val, st_val);
    return hipGetLastError();
}

}  // namespace cgmi
