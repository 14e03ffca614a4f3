/*
 * cgmi_batch.h -- many independent SPD systems, each with several right-hand
 * sides, solved by one persistent launch.
 *
 * Not part of the paper, whose solver handles one system and one right-hand
 * side (Algorithm 1): this runs Algorithm 1 independently for every pair
 * (system k, right-hand side j) -- its own alpha, beta, stop test and
 * iteration count -- with all pairs advancing inside a single kernel launch.
 * A heavy system is given a team of workgroups that owns a contiguous share
 * of its rows for the whole solve; a team synchronises through counters in
 * device memory between the phases of an iteration (q = A p with p^T q;
 * x/r update with r^T r; p update) and stops when all of its right-hand sides
 * have converged, broken down or reached maxit.  Light systems share
 * workgroups: a workgroup solves its light systems one after another, so the
 * number of systems is not bounded by the grid.  The launch is cooperative,
 * so every workgroup is resident; a wait that exceeds a time limit ends the
 * launch with CG_EDEVICE instead of hanging.
 *
 * Layout: the systems' rows are stacked (system k at row offset off[k],
 * cg_batch_layout) and every vector is row-major n_total x nrhs with the
 * right-hand sides fastest, so the nrhs values of one row are contiguous.
 *
 * Conventions as in cgmi.h: host CSR arrays are copied by cg_batch_create;
 * B and X are device pointers (float64, n_total x nrhs, 16-byte aligned when
 * two right-hand sides per lane are used); X holds the initial guess on entry
 * and the solution on return.  A stream set with
 * cg_batch_set_stream is used for every launch; cg_batch_solve blocks.
 */
#ifndef CGMI_BATCH_H
#define CGMI_BATCH_H

#include <stdint.h>

#include "cgmi.h"

#ifdef __cplusplus
extern "C" {
#endif

#define CG_BATCH_MAX_RHS 16

typedef struct cg_batch cg_batch;

/* Schedule of the persistent launch (the autotuner's search space). */
typedef struct cg_batch_sched {
    int32_t blocks_per_cu;  /* workgroups per compute unit (capped by occupancy) */
    int32_t rows_per_thread;/* rows a thread advances per step of the vector
                               phases: 1 or 2 */
    double team_exponent;   /* team size of system k proportional to n_k^team_exponent */
    int32_t max_team;       /* upper bound on a team's workgroups (0: none) */
    int32_t rhs_per_lane;   /* right-hand sides per lane: 1, or 2 (16-byte
                               loads; needs an even nrhs, else 1 is used);
                               0: 2 when nrhs is even */
    int32_t launch;         /* CG_BATCH_LAUNCH_COOPERATIVE (default): a
                               cooperative launch, whose workgroups the
                               runtime guarantees to be resident together.
                               CG_BATCH_LAUNCH_ORDINARY: an ordinary launch
                               of the same grid, for tools that cannot follow
                               cooperative launches (some profilers); the
                               grid never exceeds the kernel's occupancy, so
                               its workgroups are resident together on an
                               otherwise idle device, and a team whose
                               members never all arrive gives up after 20 s
                               (CG_EDEVICE) instead of waiting forever. */
} cg_batch_sched;

#define CG_BATCH_LAUNCH_COOPERATIVE 0
#define CG_BATCH_LAUNCH_ORDINARY 1

/* Per (system, right-hand side) outcome, index k * nrhs + j. */
typedef struct cg_batch_result {
    int32_t status;         /* CG_OK, CG_MAXIT or CG_EBREAKDOWN */
    int32_t iterations;
    double rel_res_recur;   /* sqrt(r^T r) / ||b|| of the recurrence */
    double rel_res_true;    /* ||b - A x|| / ||b|| recomputed at the end */
} cg_batch_result;

typedef struct cg_batch_stats {
    double t_kernel;        /* seconds of the persistent launch (HIP events) */
    int32_t grid;           /* workgroups launched */
    int32_t teams_multi;    /* systems whose team has more than one workgroup */
    int32_t max_team;       /* largest team */
    int32_t barriers;       /* team barriers passed by the largest team */
} cg_batch_stats;

/* nsys >= 1 systems (n[k] rows, nnz[k] entries, CSR with local column
 * indices) and nrhs right-hand sides each (1 <= nrhs <= CG_BATCH_MAX_RHS).
 * nsys may exceed the workgroups of one launch (light systems share
 * workgroups); the stacked row count and entry count must fit int32. */
int cg_batch_create(int32_t nsys, const int32_t *n, const int64_t *nnz,
                    const int32_t *const *row_ptr, const int32_t *const *col,
                    const double *const *val, int32_t nrhs, cg_batch **out);
void cg_batch_destroy(cg_batch *b);
int cg_batch_set_stream(cg_batch *b, void *hip_stream);

/* Row offsets of the systems in the stacked vectors (host, nsys + 1). */
int cg_batch_layout(const cg_batch *b, int64_t *row_offset);

void cg_batch_default_sched(cg_batch_sched *s);
int cg_batch_set_sched(cg_batch *b, const cg_batch_sched *s);
int cg_batch_get_sched(const cg_batch *b, cg_batch_sched *s);

/* Solve all pairs to ||r|| < tol ||b|| (tol = 0: exactly maxit iterations
 * each).  res: host, nsys * nrhs entries (may be NULL); stats may be NULL.
 * Returns CG_OK when every pair converged, CG_MAXIT when some pair did not
 * (none broke down), CG_EBREAKDOWN when some pair broke down. */
int cg_batch_solve(cg_batch *b, const double *B, double *X, double tol, int32_t maxit,
                   cg_batch_result *res, cg_batch_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* CGMI_BATCH_H */
