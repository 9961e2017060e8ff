// Static device scratch of the allocation-free apply (fpde_apply_noalloc).
//
// `scratch` is a file-scope device array.  In host code its name is only a
// host-side stand-in: the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current and
// kept per device; every use on the host (kernel arguments, fills) goes
// through that address.  Every call on one GPU shares that GPU's copy, so
// calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "fpde_device.h"

namespace fpde {

namespace {
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the current device's scratch (looked up on the first call per device).
hipError_t scratch_address(void** out) {
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// p[0, n) = 0 (32-bit words): tickets and coefficient sums that must start at zero
FPDE_KERNEL void k_zero_words(int64_t n, uint32_t* p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_zero_words(int64_t n, uint32_t* p, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_words, dim3(grid1(n)), dim3(256), 0, st, n, p);
    return hipGetLastError();
}

}  // namespace fpde
