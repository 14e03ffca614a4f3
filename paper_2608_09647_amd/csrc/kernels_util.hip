// kernels_util.hip -- a plain streaming copy (gfx950), the achievable-bandwidth
// reference the SpMV is reported against next to the HBM specification, and
// a plain random gather, the reference for SpMVs bound by gathers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "util_internal.h"

namespace cgmi {

namespace {

// 16-byte vector type that stays in registers (an array of HIP's double2
// with conditional stores went to scratch memory)
typedef double dbl2v __attribute__((ext_vector_type(2)));

// dst = src over n doubles.  VEC: both 16-byte aligned, so pairs move as
// 16-byte accesses.  Each workgroup copies one contiguous chunk, eight
// 16-byte pairs per thread in flight (for 1 GiB copies this beat a
// grid-stride sweep of the whole array by about a fifth: 5.3 against
// 4.3-4.5 TB/s); the odd last element, if any, goes separately.
template <bool VEC>
__global__ __launch_bounds__(256) void k_stream_copy(const double *__restrict__ src, double *__restrict__ dst,
                                                     int64_t n) {
    constexpr int U = 8;
    if constexpr (VEC) {
        const int64_t n2 = n >> 1;
        const dbl2v *s2 = reinterpret_cast<const dbl2v *>(src);
        dbl2v *d2 = reinterpret_cast<dbl2v *>(dst);
        const int64_t per = (n2 + gridDim.x - 1) / gridDim.x;
        const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n2 ? lo + per : n2;
        for (int64_t b = lo + threadIdx.x; b < hi; b += U * 256) {
            dbl2v v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (b + u * 256 < hi) v[u] = s2[b + u * 256];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (b + u * 256 < hi) d2[b + u * 256] = v[u];
        }
        if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) dst[n - 1] = src[n - 1];
    } else {
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
    }
}

// dst[i] = src[idx[i]]: random 8-byte gathers at the rate the memory
// system allows them.  Each thread takes 8 consecutive entries (two 16-byte
// index loads, 8 gathers in flight, four 16-byte stores); the chunk loop
// strides over the grid; the last n mod 8 entries go one per thread.  VEC:
// idx and dst 16-byte aligned.
template <bool VEC>
__global__ __launch_bounds__(256) void k_gather_ref(const double *__restrict__ src, const int32_t *__restrict__ idx,
                                                    double *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if constexpr (VEC) {
        const int64_t n8 = n >> 3;
        const int4 *i4 = reinterpret_cast<const int4 *>(idx);
        dbl2v *d2 = reinterpret_cast<dbl2v *>(dst);
        for (int64_t c = t0; c < n8; c += stride) {
            const int4 a = i4[2 * c], b = i4[2 * c + 1];
            const double v0 = src[a.x], v1 = src[a.y], v2 = src[a.z], v3 = src[a.w];
            const double v4 = src[b.x], v5 = src[b.y], v6 = src[b.z], v7 = src[b.w];
            d2[4 * c] = dbl2v{v0, v1};
            d2[4 * c + 1] = dbl2v{v2, v3};
            d2[4 * c + 2] = dbl2v{v4, v5};
            d2[4 * c + 3] = dbl2v{v6, v7};
        }
        for (int64_t i = (n8 << 3) + t0; i < n; i += stride) dst[i] = src[idx[i]];
    } else {
        for (int64_t i = t0; i < n; i += stride) dst[i] = src[idx[i]];
    }
}

}  // namespace

hipError_t launch_gather_ref(const double *src, const int32_t *idx, double *dst, int64_t n, int grid,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const bool vec = (((uintptr_t)idx | (uintptr_t)dst) & 15) == 0;
    if (vec)
        hipLaunchKernelGGL(k_gather_ref<true>, dim3(grid), dim3(256), 0, s, src, idx, dst, n);
    else
        hipLaunchKernelGGL(k_gather_ref<false>, dim3(grid), dim3(256), 0, s, src, idx, dst, n);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const double *src, double *dst, int64_t n, int grid, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const bool vec = (((uintptr_t)src | (uintptr_t)dst) & 15) == 0;
    if (vec)
        hipLaunchKernelGGL(k_stream_copy<true>, dim3(grid), dim3(256), 0, s, src, dst, n);
    else
        hipLaunchKernelGGL(k_stream_copy<false>, dim3(grid), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace cgmi
