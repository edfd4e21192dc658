// The single arithmetic form of one Yee component update, shared by every
// kernel schedule so that all schedules produce the same bits.
//
// Eq. 2 (Sec. 2) with cubic cells: a component f advances by its
// coefficient (dt/eps or dt/mu, with 1/dx folded in) times the difference of
// two staggered one-cell differences:
//   f_new = f + c * ((a1 - a0) - (b1 - b0))
// evaluated as one fused multiply-add after the two differences.
#pragma once

#include <hip/hip_runtime.h>

namespace fdtd {

__device__ __forceinline__ float curl_update(float f, float c, float a1, float a0, float b1, float b0)
{
    return __builtin_fmaf(c, (a1 - a0) - (b1 - b0), f);
}

__device__ __forceinline__ double curl_update(double f, double c, double a1, double a0, double b1, double b0)
{
    return __builtin_fma(c, (a1 - a0) - (b1 - b0), f);
}

}  // namespace fdtd
