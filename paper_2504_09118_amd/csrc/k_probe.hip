// Bandwidth probe: a plain streaming copy with 16-byte accesses. It moves a
// known number of bytes, so its time gives the achievable HBM bandwidth of
// the device and its memory counters calibrate those of the solver kernels.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fdtd.h"

namespace {

constexpr int kBlock = 1024;
constexpr int kUnroll = 4;

// Grid-stride copy, four 16-byte loads in flight per thread before the stores.
__global__ void __launch_bounds__(kBlock) k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n)
{
    const size_t T = (size_t)gridDim.x * kBlock;
    size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x;
    for (; q + (kUnroll - 1) * T < n; q += kUnroll * T) {
        uint4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = src[q + u * T];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) dst[q + u * T] = v[u];
    }
    for (; q < n; q += T) dst[q] = src[q];
}

}  // namespace

extern "C" int fdtd_probe_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    if (!dst || !src || bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
        return FDTD_E_ARG;
    const size_t n = bytes / 16;
    // 64 workgroups of 1024 threads per CU on 256 CUs: the fastest of the launch shapes
    // swept on MI355X (256..1024 threads, 4..64 groups per CU, 1 or 4 loads in flight)
    const unsigned grid = 256 * 64;
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, (const uint4 *)src, (uint4 *)dst,
                       n);
    return hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_E_DEVICE;
}
