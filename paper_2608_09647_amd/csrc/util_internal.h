// util_internal.h -- launchers of the streaming copy and the random gather
// (kernels_util.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cgmi {

// dst = src over n doubles (a plain streaming copy: the achievable-bandwidth
// reference); any alignment, 16-byte pairs when both are aligned.
hipError_t launch_stream_copy(const double *src, double *dst, int64_t n, int grid, hipStream_t s);
// dst[i] = src[idx[i]] for i < n (the achievable-gather reference); the
// indices are not checked.
hipError_t launch_gather_ref(const double *src, const int32_t *idx, double *dst, int64_t n, int grid,
                             hipStream_t s);

}  // namespace cgmi
