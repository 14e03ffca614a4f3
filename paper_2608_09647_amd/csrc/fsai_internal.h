// Internals of the learned FSAI preconditioner shared by kernels_fsai.hip
// and fsai.cpp: network dimensions, the parameter layout, stencil slots and
// the launch wrappers.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace cgmi {

constexpr int kFeat = 12;      // features per row
constexpr int kFeatPad = 16;   // stored features per row (bfloat16; 12..15 are 0)
constexpr int kHidden = 64;
constexpr int kOut = 5;        // outputs C, W, E, S, N
constexpr int kOutPad = 8;     // stored outputs per row (float32)
constexpr int kSlots = 5;      // stencil slots per row of A
constexpr int kSlotC = 0, kSlotW = 1, kSlotE = 2, kSlotS = 3, kSlotN = 4;
constexpr double kEpsDiag = 1e-3;

// Flat float32 parameters: W1 (64 x 12), b1, W2 (64 x 64), b2, W3 (5 x 64), b3.
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHidden * kFeat;    // 768
constexpr int kOffW2 = kOffB1 + kHidden;            // 832
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;  // 4928
constexpr int kOffW3 = kOffB2 + kHidden;            // 4992
constexpr int kOffB3 = kOffW3 + kOut * kHidden;     // 5312
constexpr int kNParams = kOffB3 + kOut;             // 5317

#if defined(__HIPCC__)
#define CGMI_HD __host__ __device__
#else
#define CGMI_HD
#endif

// Slot of column c in row i of a 5-point operator in x-fastest order.
CGMI_HD inline int stencil_slot(int64_t i, int64_t c) {
    return c == i ? kSlotC : c == i - 1 ? kSlotW : c == i + 1 ? kSlotE : c < i ? kSlotS : kSlotN;
}

// Per row i (thread per row): slot columns scol[i][5] (-1 absent), A_hat
// values sval[i][5] (C slot 1), diag[i], bfloat16 features feats[i][16].
// *err counts rows that are not 5-point or have a non-positive diagonal (own
// or neighbour's).  Row pointers may be rebased; columns are local.
hipError_t fsai_prepare(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
                        int32_t *scol, float *sval, double *diag, uint16_t *feats, int32_t *err,
                        hipStream_t s);

// Network outputs out[row][8] (0..4 valid, 5..7 zero) for the listed 16-row
// tiles (tiles[t] = first row; rows >= nrows are skipped); dg_zero[row][3]
// of the same rows is set to 0.
hipError_t fsai_forward_outputs(int32_t ntiles, const int32_t *tiles, int64_t nrows,
                                const uint16_t *feats, const float *theta, float *out, int64_t *dg_zero,
                                hipStream_t s);

// Inference for all n rows: G values into gval (CSR of tril(A); gpos[i][3]
// = positions of the C, W, S entries of row i, -1 absent) and G^T values into
// gtval[tpos[p]].
hipError_t fsai_forward_factor(int32_t n, const uint16_t *feats, const float *theta,
                               const int32_t *scol, const double *diag, const int32_t *gpos,
                               const int32_t *tpos, double *gval, double *gtval, hipStream_t s);

// Loss terms and dL/dG~ (dg[row][3]: C, W, S; 64-bit fixed point in units of
// 2^-40, accumulated with integer atomics, so the sums are reproducible) of
// the sampled rows, one wavefront per sample; partials[block] = sum of
// squared entries of E, fsai_loss_blocks(nsamp) of them.
inline int32_t fsai_loss_blocks(int32_t nsamp) {
    const int32_t b = (nsamp + 3) / 4;
    return b < 1 ? 1 : b > 2048 ? 2048 : b;
}
hipError_t fsai_loss(int32_t nsamp, const int32_t *samp_row, const int64_t *samp_base,
                     const int32_t *samp_n, const float *out, const int32_t *scol, const float *sval,
                     int64_t *dg, float coef, double *partials, hipStream_t s);

// Parameter gradient of the listed 16-row tiles: gpart[block][kNParams].
// dL/do of a row is formed from dL/dG~ (dg), the outputs and the slot table.
hipError_t fsai_backward(int32_t ntiles, const int32_t *tiles, const uint16_t *feats, const float *theta,
                         const float *out, const int64_t *dg, const int32_t *scol, float *gpart, int32_t grid,
                         hipStream_t s);

// Sum of nparts gradient partials (in order) into grad_out (may be null);
// with t_step >= 1 an Adam step on theta (m, v: moments).
hipError_t fsai_adam(int32_t nparts, const float *gpart, float *theta, float *m, float *v,
                     float *grad_out, int32_t t_step, float lr, hipStream_t s);

// Copy CSR values into the slot-major sliced layout (slices of 64 rows).
hipError_t sell_refresh(int32_t m, int32_t ntiles, const int32_t *rp, const int32_t *sell_off,
                        const double *val, double *sell_val, hipStream_t s);

// Copy CSR values into the stencil-slice layout: the k-th entry of row i goes
// to the slot of the k-th set bit of the row's mask (columns ascend, and so do
// the slice's offsets).
hipError_t stencil_refresh(int32_t m, int32_t ntiles, const int32_t *rp, const int32_t *st_off,
                           const uint8_t *st_mask, const double *val, double *st_val, hipStream_t s);

}  // namespace cgmi
