// scratch.hip -- the library's static device scratch for the entry point
// that allocates nothing (cg_solve_noalloc), and the kernel that initialises
// a solver state in device memory without a host staging copy.
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy, at its own address, until the process ends.  Host code never
// passes the array's name to a kernel or a copy (on the host it is only a
// stand-in for the device symbol); it asks once per device, with that device
// current, for the array's device address and uses that.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "cgmi_internal.h"

namespace cgmi {

namespace {

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

__global__ void k_state_init(DevState *st, double tol, int32_t maxit, double delta) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    DevState s{};
    s.tol = tol;
    s.maxit = maxit;
    s.delta = delta;
    *st = s;
}

}  // namespace

hipError_t scratch_setup() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[dev] || g_err[dev] != hipSuccess) return g_err[dev];
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && !p) e = hipErrorInvalidSymbol;
    if (e == hipSuccess) g_ptr[dev] = p;
    else g_err[dev] = e;
    return e;
}

hipError_t scratch_region(int dev, void **ptr, size_t *bytes) {
    *ptr = nullptr;
    *bytes = 0;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) return g_err[dev] != hipSuccess ? g_err[dev] : hipErrorNotInitialized;
    *ptr = g_ptr[dev];
    *bytes = kScratchBytes;
    return hipSuccess;
}

hipError_t launch_state_init(DevState *st, double tol, int32_t maxit, double delta, hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, tol, maxit, delta);
    return hipGetLastError();
}

}  // namespace cgmi
