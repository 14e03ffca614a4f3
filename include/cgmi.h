/*
 * cgmi.h -- C ABI of the MI355X sparse conjugate-gradient library (libcgmi.so).
 *
 * The library runs the hot path of the paper's sparse CG (Section 3):
 * CSR SpMV q = A p with the fused p^T q dot (Section 3.3), the fused
 * x += alpha p, r -= alpha q, r^T r update, and p = r + beta p
 * (Algorithm 1).  A contiguous block of rows [row_begin, row_end) runs on the
 * GPU; the remaining rows (the host complement) run on host threads, and the
 * shared search direction p is made visible to both sides every iteration by
 * explicit copies, or held once in mapped host memory or managed memory
 * (Section 3.2 row split, Section 3.4 memory execution modes).
 *
 * Conventions for every entry point
 *   - Matrices: CSR, int32 row pointers and column indices, float64 values,
 *     square n x n, row_ptr[0] == 0, row_ptr non-decreasing, row_ptr[n] == nnz,
 *     0 <= col < n, columns strictly increasing inside each row.  Passed as
 *     HOST pointers, borrowed only for the duration of the call: the library
 *     copies what it needs.
 *   - Vectors (b, x, y): n float64 values owned by the caller: DEVICE
 *     pointers on the handle's device (for example torch.cuda tensors) by
 *     default, HOST pointers with cg_opts.vectors = CG_VECTORS_HOST.
 *   - Work is ordered on the handle's HIP stream (cg_set_stream; default:
 *     the null stream).  Calls that say "blocking" return after the stream
 *     has drained the work they queued.
 *   - Return codes: CG_OK (0) success / converged, CG_MAXIT (1) the
 *     iteration limit was reached (not an error; x holds the last iterate),
 *     negative values are errors; cg_last_error() returns a message for the
 *     last error on the calling thread.
 *   - A handle may be used by one host thread at a time.
 */
#ifndef CGMI_H
#define CGMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CG_OK = 0,
    CG_MAXIT = 1,
    CG_EINVAL = -1,      /* bad argument or malformed CSR                        */
    CG_ENOMEM = -2,      /* host or device allocation failed                     */
    CG_EDEVICE = -3,     /* a HIP call failed                                    */
    CG_EBREAKDOWN = -4   /* p^T q <= 0 or not finite (matrix not SPD, NaN input) */
};

enum { CG_PREC_FP64 = 0, CG_PREC_MIXED = 1 };         /* cg_opts.precision */
enum { CG_PC_NONE = 0, CG_PC_FSAI = 1 };              /* cg_opts.precond   */
enum {                                                /* cg_opts.exchange  */
    CG_EXCHANGE_WHOLE = 0,
    CG_EXCHANGE_HALO = 1,
    CG_EXCHANGE_MAPPED = 2,
    CG_EXCHANGE_MANAGED = 3
};

typedef struct cg_handle cg_handle;

/* Solver options (cg_set_opts).  cg_default_opts() fills the defaults. */
typedef struct cg_opts {
    int32_t precision;     /* CG_PREC_FP64: float64 CG (Algorithm 1).
                              CG_PREC_MIXED: float32 inner CG; the true residual
                              b - A x, its norm and x stay float64 (reliable
                              updates).  GPU-only handles.                       */
    int32_t precond;       /* CG_PC_NONE, or CG_PC_FSAI: M^-1 = G^T G with the
                              factor installed by cg_set_fsai.  GPU-only.        */
    int32_t exchange;      /* how p is made visible to the GPU and the host
                              (Section 3.4 memory execution modes).
                              CG_EXCHANGE_WHOLE: separate host and device
                              copies; the whole GPU-owned / host-owned segments
                              are copied each iteration (explicit copy).
                              CG_EXCHANGE_HALO: explicit copy of only the
                              entries the other side's rows read.
                              CG_EXCHANGE_MAPPED: one copy of p in page-locked,
                              coherent host memory; kernels read and write it
                              through its device address, host threads through
                              its host address; nothing is copied.
                              CG_EXCHANGE_MANAGED: one copy of p in managed
                              memory (hipMallocManaged), used in place by both
                              sides; CG_EINVAL where the device reports no
                              managed-memory support.
                              MAPPED and MANAGED hold p in that memory for
                              GPU-only handles too (then the single-workgroup
                              path, which keeps p in LDS, is not used); they
                              need CG_PREC_FP64 and CG_PC_NONE.  cg_set_opts
                              allocates the shared p when the mode is chosen. */
    int32_t host_threads;  /* host complement threads (0: all available)        */
    int32_t check_every;   /* GPU-only: iterations queued between host polls of
                              the device convergence flag (>= 1)                */
    int32_t profile;       /* P >= 1: time the SpMV launch of every P-th
                              iteration of a GPU-only cg_solve with HIP events
                              (cg_result.t_spmv / n_spmv over those launches;
                              an event pair costs a few microseconds of stream
                              time, so a sparse sample disturbs the solve
                              less); on the single-workgroup path the pair
                              brackets the one launch of the whole solve
                              (n_spmv = 1); 0: off                               */
    int32_t small_path;    /* 1 (default): systems that fit one workgroup's LDS
                              run the whole solve in one single-workgroup kernel */
    int32_t spmv_grid;     /* workgroups of the SpMV kernels (0: automatic)      */
    int32_t spmv_kind;     /* SpMV tiling: 0 automatic, 1 vector CSR row-length
                              bins (L lanes per row), 2 stream tiles (runs of
                              at most 64 rows with at most 509 nonzeros,
                              loaded flat, 8 gathers in flight per lane; used
                              only when every row fits, else 1), 3 sliced
                              tiles (64-row slices
                              stored slot-major, one lane per row; rows of at
                              most 64 nonzeros, else 1), 4 dictionary-sliced
                              tiles (the sliced layout with a 4-bit index per
                              slot into a per-slice table of at most 15 column
                              offsets; rows of at most 8 nonzeros, else 3),
                              5 column blocks (one accumulating pass per block
                              of spmv_colblock columns, so gathers from p stay
                              in the L2; each pass on stream tiles when every
                              row's entries in the block fit one, else rows
                              in natural order with lanes for half the
                              block's mean row length, or length bins when a
                              block has a row over 4096 entries; for
                              scattered columns),
                              6 stencil slices (slot j of a 64-row slice holds
                              the entries at the slice's j-th column offset, so
                              columns are row + a slice-uniform offset and a
                              byte per row marks the present slots; rows of at
                              most 8 nonzeros, at most 8 distinct offsets per
                              slice, float64; else 4),
                              7 gap-coded slices (the sliced layout of 3 with
                              each row's first column as int32 and every
                              further column as its gap to the previous one
                              in 16 bits (all SpMV modes, float64 and
                              float32); rows of at most 8 nonzeros whose
                              consecutive columns lie at most 65,536 apart;
                              else 3).
                              Automatic picks 5 when more than half of the
                              entries lie farther than 262,144 columns from the
                              diagonal and the vector spans at least two blocks,
                              else 6 where it applies, else 4 when rows have
                              <= 8 nonzeros and every slice fits the table,
                              else 7 where it applies, else 3 when rows have
                              <= 64 nonzeros and slicing pads by <= 25%,
                              else 2 where every row fits a run and the
                              block has >= 262,144 rows of mean length <= 64
                              or >= 131,072 of mean length <= 32, else 1.     */
    int32_t spmv_colblock; /* columns per block of the column-blocked tiling
                              (spmv_kind 5); 0: 262,144 (2 MB of float64 p)     */
    double refine_delta;   /* mixed precision: a float64 refinement is made
                              when the float32 residual drops by this factor    */
    int32_t vectors;       /* CG_VECTORS_DEVICE (default): b, x, y of cg_spmv
                              and cg_solve are device pointers.
                              CG_VECTORS_HOST: they are host pointers; the
                              library copies them to device buffers of its
                              own (allocated on first use, n float64 each for
                              b / x and x / y), runs the device path and
                              copies the result back before returning (both
                              calls then block).  cg_solve_noalloc takes
                              device pointers only.                             */
    int32_t fuse_dir;      /* GPU-only float64 solves whose A sits in stencil
                              slices (spmv_kind 6): CG_FUSE_ON runs the
                              direction update p = r + beta p (preconditioned:
                              z + beta p) and the x update it carries inside
                              the next iteration's SpMV, each gathered p entry
                              formed on the fly (Algorithm 1's steps
                              unchanged: the same operations on the same
                              operands, so x, r, p and every reduction are
                              bitwise those of separate kernels; it saves a
                              launch and a pass over p, but gathers r as well
                              as p); CG_FUSE_OFF: separate kernels;
                              CG_FUSE_AUTO (default): fused for
                              preconditioned solves of at most 2,097,152 GPU
                              rows and plain ones of at most 262,144 (where
                              the launch and pass it saves outweigh the extra
                              gathers), separate above.                        */
} cg_opts;

enum { CG_VECTORS_DEVICE = 0, CG_VECTORS_HOST = 1 };  /* cg_opts.vectors   */
enum { CG_FUSE_AUTO = 0, CG_FUSE_ON = 1, CG_FUSE_OFF = 2 };  /* cg_opts.fuse_dir */

/* Per-solve record.  Times in seconds.  Fields follow the per-pass record of
 * Section 4.1: solve time, iterations, convergence, residuals, CPU compute
 * time, GPU task time, barrier time and D2H / H2D copy times; rows and
 * nonzeros per side follow Section 3.2. */
typedef struct cg_result {
    int32_t status;          /* same value as the return code                    */
    int32_t iterations;      /* CG iterations (SpMVs inside the loop)            */
    int32_t converged;       /* 1 if the stop test was met                       */
    int32_t fp64_residuals;  /* mixed precision: float64 residuals formed        */
    double rel_res_recur;    /* sqrt(rho)/||b|| of the recurrence at exit        */
    double rel_res_true;     /* ||b - A x|| / ||b|| recomputed after the solve   */
    double t_solve;          /* wall time of the solve                           */
    double t_gpu;            /* GPU kernel time (split mode: summed per phase)   */
    double t_cpu;            /* host complement compute time                     */
    double t_barrier;        /* time waiting at CPU/GPU synchronisation points  */
    double t_d2h, t_h2d;     /* p exchange copy times                            */
    double t_spmv;           /* summed SpMV kernel time (opts.profile)           */
    int32_t n_spmv;          /* SpMV launches timed                              */
    int32_t rows_gpu, rows_cpu;
    int64_t nnz_gpu, nnz_cpu;
    int32_t fell_back;       /* 1 if a preconditioned / mixed solve fell back to
                                plain float64 CG                                 */
    int32_t spmv_kind;       /* SpMV tiling used on the GPU rows: 1 vector bins,
                                2 stream tiles, 3 sliced tiles, 4 dictionary-
                                sliced tiles, 5 column blocks, 6 stencil slices,
                                7 gap-coded slices (0: no GPU rows)              */
    int32_t fused_dir;       /* 1 if the direction update ran inside the SpMV
                                (cg_opts.fuse_dir)                               */
} cg_result;

/* Create a solver for the n x n CSR matrix (host arrays, copied).  Rows
 * [row_begin, row_end) go to the GPU, the others to host threads
 * (Section 3.2: n_gpu = round(g n) gives [0, n_gpu)); row_begin == row_end
 * means host only, [0, n) GPU only.  Validates the CSR (CG_EINVAL with a
 * message on failure).  Uploads the GPU row block with its row pointers
 * rebased to start at 0 (the matrix is read-only and never re-sent). */
int cg_create(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
              const double *val, int32_t row_begin, int32_t row_end, cg_handle **out);

/* Release every host and device resource of h.  NULL is a no-op. */
void cg_destroy(cg_handle *h);

/* Order the handle's work on this HIP stream (a hipStream_t; NULL = null
 * stream).  The library also creates private streams for p exchange. */
int cg_set_stream(cg_handle *h, void *hip_stream);

void cg_default_opts(cg_opts *o);
int cg_set_opts(cg_handle *h, const cg_opts *o);
int cg_get_opts(const cg_handle *h, cg_opts *o);

/* y = A x (Section 3.1, q_i = sum_j A_ij p_j) for all n rows.  x, y: n
 * float64 each (device pointers, or host pointers with CG_VECTORS_HOST), must
 * not overlap.  GPU-only handles with device vectors: queued on the stream
 * and returns at once.  Otherwise blocking (the host rows are computed on
 * host threads from a copy of x). */
int cg_spmv(cg_handle *h, const double *x, double *y);

/* y = A32 x in float32 (the inner SpMV of mixed precision): float32 copies
 * of the values, float32 x (device, n), float32 y (device, n); each row summed
 * in float32.  GPU-only handles with cg_opts.precision = CG_PREC_MIXED set
 * (which builds the float32 copies); CG_EINVAL otherwise.  Queued on the
 * stream. */
int cg_spmv_f32(cg_handle *h, const float *x, float *y);

/* Solve A x = b by CG (Algorithm 1): x (in/out; device, or host with
 * CG_VECTORS_HOST) holds the initial guess and receives the last iterate.  Stops at the top of an iteration when
 * sqrt(r^T r) < tol * ||b||_2 (tol = 0: fixed work of maxit iterations).
 * b == 0 gives x = 0.  Blocking.  res (may be NULL) receives the record.
 * Returns CG_OK, CG_MAXIT, CG_EBREAKDOWN or an error. */
int cg_solve(cg_handle *h, const double *b, double *x, double tol, int32_t maxit,
             cg_result *res);

/* cg_solve for callers that cannot allocate memory while solving (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results as cg_solve on a
 * GPU-only handle with CG_PREC_FP64, CG_PC_NONE and p in device memory
 * (CG_EINVAL for any other handle or option), but every work buffer (the
 * working x, r, q, two p buffers, the partial sums and the solver state)
 * lives in one static device array of the library, CG_NOALLOC_SCRATCH_BYTES
 * per device, held by each device the library runs on until the process
 * ends.  Nothing is allocated: no hipMalloc / hipFree, no pinned host
 * memory, no events (cg_opts.profile is ignored; t_spmv and n_spmv stay 0).
 * The array holds five vectors of n + 2 float64 values (each rounded up to
 * 256 bytes), 4 x 16 float64 partial sums per compute unit and the state:
 * on a 256-CU MI355X n is at most 1,674,430 rows; a larger n returns
 * CG_EINVAL with the limit in cg_last_error().  The scratch keeps the last call's contents; the solver
 * state in it is re-initialised by every call.  All calls on one device share
 * the one array: calls that overlap in time on the same device (two host
 * threads, or two streams) race and must be serialised by the caller.  Its
 * device address is looked up once per device when the first handle is
 * created there.  Blocking, like cg_solve. */
#define CG_NOALLOC_SCRATCH_BYTES (64u << 20)
int cg_solve_noalloc(cg_handle *h, const double *b, double *x, double tol, int32_t maxit,
                     cg_result *res);

/* Bit-exact readback of the GPU row block as uploaded: rows + 1 rebased row
 * pointers, nnz_gpu columns and values (host buffers sized by the caller from
 * cg_result / cg_slice_info).  For checking the row split. */
int cg_slice_info(const cg_handle *h, int32_t *rows_gpu, int64_t *nnz_gpu);
int cg_read_slice(const cg_handle *h, int32_t *row_ptr, int32_t *col_idx, double *val);

/* dst = src over n float64 values on the current device (device pointers,
 * any alignment, must not overlap): a plain streaming copy, the achievable
 * HBM bandwidth the SpMV's rate is reported against next to the
 * specification.  Queued on hip_stream (a hipStream_t; NULL = null stream).
 * CG_EINVAL for NULL pointers with n > 0 or n < 0. */
int cg_hbm_copy(const double *src, double *dst, int64_t n, void *hip_stream);

/* dst[i] = src[idx[i]] for i < n on the current device (device pointers;
 * idx int32; dst must not overlap src or idx): a plain random gather, eight
 * 8-byte gathers in flight per thread, the achievable rate of gathers an
 * SpMV with scattered columns is reported against (e.g. from a src that
 * fits the L2 or the last-level cache).  Every idx[i] must lie in the src
 * allocation: the indices are not checked on the device.  Queued on
 * hip_stream.  CG_EINVAL for NULL pointers with n > 0 or n < 0. */
int cg_gather(const double *src, const int32_t *idx, double *dst, int64_t n, void *hip_stream);

/* Message for the last error on this thread ("" if none). */
const char *cg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CGMI_H */
