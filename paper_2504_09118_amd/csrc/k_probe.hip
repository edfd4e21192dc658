// Bandwidth probe: a plain streaming copy with 16-byte accesses. It moves a
// known number of bytes, so its time gives the achievable HBM bandwidth of
// the device and its memory counters calibrate those of the solver kernels.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fdtd.h"

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x; q < n; q += stride)
        dst[q] = src[q];
}

}  // namespace

extern "C" int fdtd_probe_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    if (!dst || !src || bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
        return FDTD_E_ARG;
    const size_t n = bytes / 16;
    const unsigned grid = 256 * 32;  // 32 workgroups per CU on 256 CUs
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, (const uint4 *)src, (uint4 *)dst,
                       n);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_E_DEVICE;
}
