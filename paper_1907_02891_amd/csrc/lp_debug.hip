// Debug fill for LP_DEBUG_POISON: a quiet NaN over a workspace region before
// a call, so that any element a stage reads before some stage has written it
// turns the output into NaN (a plain kernel, not a memset, so that it can sit
// in a captured graph).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lp {

namespace {

__global__ void __launch_bounds__(256) k_poison(uint32_t *__restrict__ p, size_t n)
{
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = 0x7fc0deadu;  // a quiet NaN
}

}  // namespace

// bytes: a multiple of 4 (workspace regions are 256-byte aligned)
hipError_t launch_poison(void *p, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_poison, dim3(static_cast<unsigned>(blocks < 8192 ? blocks : 8192)), dim3(256), 0, s,
                       static_cast<uint32_t *>(p), n);
    return hipGetLastError();
}

}  // namespace lp
