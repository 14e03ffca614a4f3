// Internal interface between the host runtime (cgmi.cpp, built by g++) and
// the HIP kernels (*.hip, built by hipcc for gfx950).  Plain structs only.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#if defined(__HIPCC__)
#define CGMI_HD __host__ __device__
#else
#define CGMI_HD
#endif

namespace cgmi {

constexpr int kBlock = 256;     // threads per workgroup of the streaming kernels
constexpr int kWaveSize = 64;   // CDNA wavefront
constexpr int kMaxBins = 8;     // lanes-per-row classes 1,2,4,...,64
constexpr int kHugeRow = 4096;  // longer rows are reduced by a whole workgroup

// Device-resident solver state.  Each field is written by one workgroup
// (workgroup 0) of one kernel and read by later kernels or by the host; the
// coefficient history is double-buffered by iteration parity so a kernel
// never reads a value its own grid is writing.
struct DevState {
    double rho[2];     // rho_k = r_k^T r_k (or r^T z) by iteration parity
    double bb;         // b^T b
    double tol;        // relative tolerance
    double pq;         // last p^T q (diagnostics)
    double rr;         // last r^T r
    double delta;      // mixed precision: refinement factor
    double rmax;       // mixed precision: residual norm at the last refinement
    int32_t iter;      // completed iterations
    int32_t maxit;
    int32_t done;      // 0 running, 1 converged, 2 iteration limit, 3 breakdown
    int32_t nrefine;   // mixed precision: float64 residuals formed
    double rr_true;    // single-workgroup solve: ||b - A x||^2 of the returned x
    double alpha_prev; // two-iteration x update: alpha of the last even iteration
    int32_t r_iter;    // device-coefficient paths: k + 1 once r of iteration k is
                       // updated (the deferred x update of iteration k runs only
                       // then; it never reads `done`, which its own workgroup 0
                       // may set while other workgroups have yet to start)
    int32_t spmv_iter; // fused direction update: the last iteration whose SpMV ran
};

enum { kDoneRunning = 0, kDoneConverged = 1, kDoneMaxit = 2, kDoneBreakdown = 3, kDoneRefine = 4 };

// One class of rows processed with the same number of lanes per row.
struct Bin {
    int32_t lanes;        // 1..64 lanes per row
    int32_t first;        // first position in the row list
    int32_t count;        // rows in the bin
    int32_t tile_begin;   // first wavefront tile of the bin (numbered over all bins)
};

// Stream tiles (kind kTileStream): runs of at most 64 consecutive rows per
// wavefront tile (first rows in tile_row) whose nonzeros are loaded flat by
// the wavefront in 16-byte groups counted from the tile's first nonzero
// rounded down to a multiple of 4; a run fits when (k0 mod 4) + nnz(run) <=
// kStreamNnz.  col/val allocations carry kStreamNnz padding entries (column
// 0, value 0).
constexpr int kStreamPerLane = 8;
constexpr int kStreamNnz = kWaveSize * kStreamPerLane;
// Sliced tiles (kind kTileSliced): the block is re-laid out in slices of 64
// rows stored slot-major (slot j of every row of the slice, then slot j+1,
// ...), padded to the slice's longest row; slice t starts at sell_off[t].
constexpr int kSliceMaxWidth = 8;  // widths up to this take the unrolled path
// Gap-coded slices (spmv_kind 7; the sliced layout, float64 paired tiles):
// 16-bit codes in sell_gap, slot-major like the values, and one byte per row
// in sell_lenx (64 per slice): bits 0-3 the row's length, bits 4-7 bits
// 16-19 of its first-column offset.  Slot 0 of a row holds bits 0-15 of that
// offset, first column minus the row's global index as a 20-bit two's
// complement number (an empty row, or a padding row of the last slice,
// starts at the block's last row); slot j >= 1 holds column j minus column
// j-1 minus 1 (0 in padding slots, which the kernel recognises by the
// length: they gather the row's last entry again and are never summed).
// Applies where rows have at most 8 entries, consecutive columns lie at most
// 2^16 apart and first columns within 2^19 of the diagonal: 2 index bytes
// per slot instead of 4.
// Dictionary-sliced tiles (kind kTileSlicedDict): the sliced layout's values
// with the columns replaced by 4 bits per slot.  Slice t keeps up to 15
// distinct column offsets (column - global row) in sell_dict[16t .. 16t+14]
// (entry 15 is 0); nibble j of sell_idx[64t + l] is the dictionary index of
// slot j of lane l's row, or kDictPad (padding: gathers the row's own entry,
// never summed).  Widths up to kSliceMaxWidth (8 nibbles) only.
constexpr int kDictSize = 16;
constexpr uint32_t kDictPad = 0xFu;
// Column-blocked tiles (kind kTileColBlocked): for matrices whose columns
// scatter over a vector larger than the L2, the entries are split by column
// block (kColBlockCols columns, about 2 MB of float64 p) into one CSR per
// block; q = A p runs as one pass per block (vector bins over the rows with
// entries in the block, q accumulated), so every pass gathers from a segment
// of p that stays in each XCD's L2.
constexpr int kMaxColBlocks = 64;
constexpr int32_t kColBlockCols = 1 << 18;
// Stencil slices (kind kTileStencil): each 64-row slice takes the sorted
// union of its rows' column offsets (column - global row), at most
// kSliceMaxWidth of them, in st_offs[8t .. 8t+7]; slot j of every row of the
// slice holds the entry at offset st_offs[8t+j] (value 0 where the row has
// none), so a slot's column is the row plus a slice-uniform offset, and bit j
// of the row's byte st_mask[64t + l] says whether the entry exists.  Slots are
// in ascending column order, so rows are summed exactly in CSR order.
// Values slot-major from st_off[t], float64 only.
enum { kTileVector = 0, kTileStream = 1, kTileSliced = 2, kTileSlicedDict = 3, kTileColBlocked = 4,
       kTileStencil = 5 };

struct Schedule {
    Bin bins[kMaxBins];
    int32_t nbins;
    int32_t ntiles;       // wavefront tiles over all bins
    int32_t identity;     // 1: the row list is 0..m-1 (no indirection)
    int32_t huge_first;   // rows longer than kHugeRow: positions in the row list
    int32_t huge_count;
    int32_t kind;         // kTileVector .. kTileStencil
    int32_t stream_nt;    // dictionary / stencil tiles: 1 = load the matrix and store q nontemporally
};

// A matrix whose streamed bytes exceed half the last-level cache (256 MB on
// MI355X) cannot stay cached across products: its loads (and the q stores)
// are issued nontemporally so that the gathered vector keeps the caches.
// Smaller matrices are re-read from the cache every iteration and keep
// ordinary loads.
constexpr int64_t kStreamNtBytes = 128ll << 20;

// Rows per group of lanes and per wavefront tile for a lanes-per-row class:
// a wavefront holds 64/lanes groups; each group takes up to 8 rows per tile
// (at most 64 rows per tile, one row pointer pair per lane).
CGMI_HD constexpr inline int rows_per_group(int lanes) {
    return lanes == 1 ? 1 : (lanes < 8 ? lanes : 8);
}
CGMI_HD constexpr inline int rows_per_wave_tile(int lanes) {
    return (kWaveSize / lanes) * rows_per_group(lanes);
}

// Matrix operand of the SpMV kernels: `m` rows with rebased row pointers;
// columns index the full length-n vector.
struct CsrDev {
    int32_t m;
    const int32_t *rp;
    const int32_t *ci;
    const double *val;
    const int32_t *rows;      // row list ordered by bin (nullptr when identity)
    const int32_t *sell_off;  // sliced layout: slice offsets (ntiles + 1)
    const int32_t *sell_ci;   //   slot-major columns
    const double *sell_val;   //   slot-major values
    const float *val32;       // float32 copies of the values (mixed precision)
    const float *sell_val32;
    const uint32_t *sell_idx; // dictionary-sliced layout: packed slot bytes
    const int32_t *sell_dict; //   per-slice column offsets
    int32_t col_base;         // global index of local row 0
    const struct ColBlocks *cb;  // column-blocked layout (host memory; launch side only)
    const int32_t *st_off;    // stencil slices: slice offsets into st_val (ntiles + 1)
    const int32_t *st_offs;   //   per-slice column offsets (8 per slice)
    const uint8_t *st_mask;   //   per-row slot bits
    const double *st_val;     //   slot-major values
    const uint8_t *sell_len;  // sliced layout: row lengths, one byte per row (64 per slice)
    const int32_t *tile_row;  // adaptive stream tiles: first row of each tile (ntiles + 1)
    const uint8_t *sell_lenx; // gap-coded slices: length and offset bits per row (64 per slice)
    const uint16_t *sell_gap; //   slot-major 16-bit column codes
};

// Per-block operands of the column-blocked tiling (kept on the host by the
// launcher; each block's CSR has all m rows, its row list only those with
// entries in the block).
struct ColBlocks {
    int32_t nb;
    CsrDev dev[kMaxColBlocks];
    Schedule sched[kMaxColBlocks];
    int32_t grid[kMaxColBlocks];
};

// Partial sums of one reduction: one value per workgroup of the kernel that
// produced them, summed in workgroup order by the consumer.
struct Partials {
    const double *v;
    int32_t count;
};

// ---- launch wrappers (kernels_cg.hip) ------------------------------------
// Every wrapper returns the hipError_t of the launch.

enum { kSpmvPlain = 0, kSpmvDot = 1, kSpmvResidual = 2, kSpmvAccum = 3, kSpmvDir = 4 };

// q = A p on the block's rows.
//   kSpmvPlain:    nothing else (with st: nothing once the solve has stopped).
//   kSpmvDot:      out_partials[wg] = sum p_own_i q_i.  With `k0_check`
//                  (first iteration of a device-driven solve) every workgroup
//                  first reduces the setup partials (r^T r in `in0`, b^T b in
//                  `in1`), applies the stop test, and workgroup 0 records
//                  rho_0, b^T b and the outcome in st.
//   kSpmvResidual: q = b - A p written to q and p_dst; out_partials[wg] =
//                  sum q_i^2, out_partials[grid + wg] = sum b_i^2.
hipError_t launch_spmv(const CsrDev &A, const Schedule &S, int grid, const double *p, double *q,
                       const double *p_own, const double *b, double *p_dst, double *out_partials,
                       Partials in0, Partials in1, DevState *st, int mode, int k0_check,
                       hipStream_t s);

// float32 SpMV (mixed precision): q32 = A32 p32 with kSpmvPlain or kSpmvDot
// (out_partials[wg] = sum of float64 products p_own_i q_i; with st, an early
// exit once the solve has stopped).  Vector-bin and sliced tilings only.
hipError_t launch_spmv_f32(const CsrDev &A, const Schedule &S, int grid, const float *p, float *q,
                           const float *p_own, double *out_partials, DevState *st, int mode,
                           hipStream_t s);

// Mixed precision vector kernels (float32 r, p, q; float64 x and sums).
//   update: alpha = rho_k / sum(pq); x += alpha p; r -= (float)alpha q;
//           out[wg] = sum r_i^2 (float64).  Breakdown as for launch_update_xr.
//   p step: rho_{k+1} = sum(rr); a refinement is requested (st->done =
//           kDoneRefine, no update) when sqrt(rho_{k+1}) < delta * rmax or
//           < tol ||b||; otherwise p = r + (float)beta p.  device_coef = 0:
//           p = r + (float)beta_arg p with no test.
//   convert: r32 = (float) r64, out[wg] = sum r32_i^2; with init, p32 = r32.
hipError_t launch_update_xr_mixed(int32_t m, int grid, double *x, float *r, const float *p,
                                  const float *q, double *out_partials, Partials pq, DevState *st,
                                  int32_t k, hipStream_t s);
hipError_t launch_update_p_mixed(int32_t m, int grid, const float *r, float *p, Partials rr,
                                 DevState *st, int device_coef, int32_t k, double beta_arg,
                                 hipStream_t s);
hipError_t launch_convert_residual(int32_t m, int grid, const double *r64, float *r32, float *p32,
                                   double *out_partials, int init_p, hipStream_t s);

// x += alpha p, r -= alpha q; out_partials[wg] = sum r_i^2.
// device_coef: alpha = rho_k / sum(pq), rho_k = st->rho[k & 1]; a breakdown
// (p^T q <= 0 or not finite) leaves x, r untouched and sets st->done.
// Otherwise alpha = alpha_arg.
hipError_t launch_update_xr(int32_t m, int grid, double *x, double *r, const double *p_own,
                            const double *q, double *out_partials, Partials pq, DevState *st,
                            int device_coef, int32_t k, double alpha_arg, hipStream_t s);

// p = r + beta p with beta from the host (split mode; the device-coefficient
// paths use launch_update_px and launch_update_p_pcg).
hipError_t launch_update_p(int32_t m, int grid, const double *r, double *p_own, double beta, hipStream_t s);

// Preconditioned CG, r update fused with t = G r_new for a factor G of at
// most `width` <= kFusedGWidth entries per row (CSR grp/gci/gval, rows
// rebased, columns < m): r_new = r_old - alpha q (another buffer than r_old),
// t = G r_new, out_partials[wg] = sum r_new_i^2; alpha = rho_k / sum(pq),
// breakdown recorded in st as by launch_update_xr.  x is updated later, by
// launch_update_p_pcg.  One row per thread: grid <= the partial buffers' size.
constexpr int kFusedGWidth = 8;
hipError_t launch_pcg_xr_g(int32_t m, int grid, int width, const int32_t *grp, const int32_t *gci,
                           const double *gval, const double *r_old, double *r_new, const double *q,
                           double *t, double *out_partials, Partials pq, DevState *st, int32_t k,
                           hipStream_t s);

// The same for a factor G in stencil slices (st_off/st_offs/st_mask/st_val as
// built for the SpMV, columns = rows + offsets): identical results; grid a
// multiple of 8, one 64-row slice per wavefront and step.
hipError_t launch_pcg_xr_gs(int32_t m, int grid, const int32_t *st_off, const int32_t *st_offs,
                            const uint8_t *st_mask, const double *st_val, const double *r_old, double *r_new,
                            const double *q, double *t, double *out_partials, Partials pq, DevState *st,
                            int32_t k, hipStream_t s);

// Preconditioned CG (z = M^-1 r): p = z + beta p, rho = r^T z from the rz
// partials, the stop test on the rr partials; first = 1 is the setup step
// (rho_0, ||b||^2 from bb, stop test at the top of iteration 0, p = z).
// x non-null (after launch_pcg_xr_g): x += alpha p first, alpha recomputed
// as there, for every iteration whose r was updated, also the last one.
// Float64 CG with device coefficients and the x update deferred to the p
// update: r -= alpha q (partials of r^T r); then x += alpha p and, unless the
// solve stops, p = r + beta p.  Vectors 16-byte aligned.
hipError_t launch_update_r(int32_t m, int grid, double *r, const double *q, double *out, Partials pq,
                           DevState *st, int32_t k, hipStream_t s);
hipError_t launch_update_px(int32_t m, int grid, double *x, const double *r, double *p, Partials rr,
                            DevState *st, int32_t k, hipStream_t s);
// The same with x updated every other iteration from two p buffers: p_k in
// p_cur, p_{k+1} written to p_oth.  Even k: p update only (x owes alpha_k
// p_k; on a stop x takes it at once); odd k: x += alpha_{k-1} p_{k-1}
// (p_oth) then alpha_k p_k, the same fmas in the same order as one update
// per iteration; after a breakdown in the r update of an odd k it adds the
// owed alpha_{k-1} p_{k-1} to x instead.
hipError_t launch_update_pxb(int32_t m, int grid, double *x, const double *r, const double *p_cur,
                             double *p_oth, Partials rr, DevState *st, int32_t k, hipStream_t s);
hipError_t launch_update_p_pcg(int32_t m, int grid, const double *z, double *p, double *x, Partials rr,
                               Partials rz, Partials bb, DevState *st, int first, int32_t k,
                               hipStream_t s);

// The direction update of iteration k fused into the SpMV of iteration k+1
// (GPU-only handles whose A sits in stencil slices): the coefficient step of
// launch_update_pxb (pcg = 0; d = r, p_oth holds p_{k-1}) or of
// launch_update_p_pcg (pcg = 1; d = z, x updated every iteration), then
// q = A p_{k+1} with p_{k+1} = d + beta p_cur formed per gathered column and
// written to p_oth, the owed x update, and out[wg] = the p^T q partial of
// workgroup wg.  At a stop only x is completed.  Bitwise the results of the
// separate kernels followed by launch_spmv(kSpmvDot) on the same grid.
// spmv_dir_applies: the tiling, grid (a multiple of 8) and 16-byte
// alignment the kernel needs; otherwise launch_spmv_dir returns
// hipErrorInvalidValue.
bool spmv_dir_applies(const CsrDev &A, const Schedule &S, int grid, const void *p_cur, const void *d,
                      const void *p_oth, const void *x, const void *q);

// With the direction update fused: did the SpMV of iteration i run?
// Iteration 0's did unless the stop test at its top ended the solve; a later
// one's (inside the launch that ended iteration i-1) iff that launch
// recorded it.
inline bool fused_spmv_ran(const DevState &s, int32_t i) {
    if (i == 0) return !(s.iter == 0 && (s.done == kDoneConverged || s.done == kDoneMaxit));
    return i <= s.spmv_iter;
}
hipError_t launch_spmv_dir(const CsrDev &A, const Schedule &S, int grid, const double *p_cur, const double *d,
                           double *p_oth, double *x, double *q, double *out, Partials rr, Partials rz,
                           DevState *st, int32_t k, int pcg, hipStream_t s);

// Whole-solve single-workgroup CG for small systems (kernels_small.hip; p
// held in LDS): reads x0 from x and writes the solution there; leaves iter,
// done, rr, bb and rr_true in st.
int small_path_max_rows();
hipError_t launch_cg_small(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
                           const double *b, double *x, double tol, int32_t maxit, DevState *st,
                           int32_t max_row_len, hipStream_t s);

// Gather / scatter of p entries for the halo exchange.
hipError_t launch_gather(int32_t cnt, const int32_t *idx, const double *src, double *dst,
                         hipStream_t s);
hipError_t launch_scatter(int32_t cnt, const int32_t *idx, const double *src, double *dst,
                          hipStream_t s);

int device_cu_count();

// The library's static device scratch (scratch.hip), used by the entry point
// that allocates nothing: kScratchBytes per device, 256-byte aligned.
// scratch_setup() looks up the array's device address for the current
// device (once per device; later calls return the first result);
// scratch_region() returns it for device `dev` after that.
constexpr size_t kScratchBytes = size_t(64) << 20;
hipError_t scratch_setup();
hipError_t scratch_region(int dev, void **ptr, size_t *bytes);
// Writes a fresh DevState (zeros, tol, maxit, delta) with a one-thread kernel.
hipError_t launch_state_init(DevState *st, double tol, int32_t maxit, double delta, hipStream_t s);

}  // namespace cgmi
