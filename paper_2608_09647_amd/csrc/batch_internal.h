// Internals of the batched persistent solve shared by kernels_batch.hip and
// batch.cpp.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace cgmi {

constexpr int kBatchThreads = 256;                  // threads per workgroup
constexpr int kBatchLanes = 16;                     // lanes per row: one per right-hand side
constexpr int kBatchRowsPerStep = kBatchThreads / kBatchLanes;
constexpr int kBatchSlots = 4;                      // partial sums per workgroup: p^T q, r^T r, b^T b, true r^T r

struct BatchOutDev {
    int32_t status;
    int32_t iterations;
    double rel_res_recur;
    double rel_res_true;
};

// Everything the persistent kernel reads; passed by value.
struct BatchArgs {
    const int32_t *rp;          // stacked CSR: row pointers (n_total + 1)
    const int32_t *ci;          // global (stacked) column indices
    const double *val;
    const double *B;            // n_total x nrhs, right-hand sides fastest
    double *X, *R, *P, *Q;
    double *part;               // [grid][kBatchSlots][kBatchLanes] partial sums
    int32_t *bar;               // [nsys] team barrier counters (0 at launch)
    int32_t *err;               // [1] set when a team wait times out
    const int32_t *wg_item;     // [grid + 1] the workgroup's items are wg_item[w] .. wg_item[w+1]-1
    const int32_t *item_sys;    // [items] system of an item
    const int32_t *item_rank;   // [items] rank of the workgroup in that system's team
    const int32_t *team_first;  // [nsys] first workgroup of the team (the hosting one for a team of one)
    const int32_t *team_size;   // [nsys]
    const int64_t *row_off;     // [nsys + 1]
    const int32_t *strip;       // [nsys] line length D of a strip-ordered phase A (0: row order)
    BatchOutDev *out;           // [nsys * nrhs]
    int32_t *episodes;          // [nsys] barriers passed (statistics)
    int32_t nrhs;
    int32_t maxit;
    double tol;
    int64_t timeout_ticks;      // wall-clock ticks a team wait may take
};

// Occupancy of the persistent kernel (workgroups per compute unit) for a
// variant: rows a thread advances per step (1, 2), right-hand sides per lane
// (1; 2 needs an even nrhs and 16-byte aligned vectors).
int batch_blocks_per_cu(int rows_per_thread, int rhs_per_lane);
// Launch of the persistent kernel over `grid` workgroups: cooperative, or
// ordinary (cooperative = 0) for a grid already checked to be resident.
hipError_t launch_batch_cg(const BatchArgs &a, int grid, int rows_per_thread, int rhs_per_lane, int cooperative,
                           hipStream_t s);

}  // namespace cgmi
