// Device-resident scratch for lp_convolve_noalloc: the intermediate spectra
// of one map live in a file-scope device array instead of the caller's
// workspace, so that a caller that cannot allocate device memory at call
// time (code under stream capture, serving loops, harnesses that forbid
// allocation) still runs the hot path.  The array is part of the library's
// code object: each GPU the library runs on holds its own copy, at its own
// address, from the first launch on that GPU until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lp_internal.h"

namespace lp {

namespace {

static __device__ __align__(256) float2 scratch[kNoAllocBytes / sizeof(float2)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

// Device address of the current device's copy of the scratch array.  The
// array's name is only a host-side handle; its device address comes from the
// runtime, looked up once per device with that device current and kept.
hipError_t noalloc_scratch(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = p;
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

}  // namespace lp
