// Field storage types and their conversions to the compute type.
//
// FP32 and FP64 fields compute in their own type. 16-bit fields (IEEE half,
// bfloat16) are widened to FP32 on load, all arithmetic of a sweep stays in
// FP32 registers and LDS, and values are rounded to nearest even once when a
// sweep stores them. A difference of two 16-bit values is exact in FP32, so
// the curl terms carry no extra rounding.
#pragma once

#include <hip/hip_runtime.h>

namespace fdtd {

// bfloat16 as raw bits (sign, 8 exponent bits, 7 fraction bits).
struct bf16 {
    unsigned short u;
};

typedef _Float16 f16;

__host__ __device__ inline float bf16_to_float(bf16 b)
{
    union {
        unsigned int u;
        float f;
    } x;
    x.u = (unsigned int)b.u << 16;
    return x.f;
}

// Round to nearest, ties to even; NaN stays a quiet NaN.
__host__ __device__ inline bf16 float_to_bf16(float f)
{
    union {
        unsigned int u;
        float f;
    } x;
    x.f = f;
    bf16 r;
    if ((x.u & 0x7fffffffu) > 0x7f800000u) {
        r.u = (unsigned short)((x.u >> 16) | 0x40u);
        return r;
    }
    const unsigned int lsb = (x.u >> 16) & 1u;
    r.u = (unsigned short)((x.u + 0x7fffu + lsb) >> 16);
    return r;
}

template <typename S>
struct Store;

template <>
struct Store<float> {
    using C = float;
    __host__ __device__ static C widen(float v) { return v; }
    __host__ __device__ static float narrow(C v) { return v; }
};

template <>
struct Store<double> {
    using C = double;
    __host__ __device__ static C widen(double v) { return v; }
    __host__ __device__ static double narrow(C v) { return v; }
};

template <>
struct Store<f16> {
    using C = float;
    __host__ __device__ static C widen(f16 v) { return (float)v; }
    __host__ __device__ static f16 narrow(C v) { return (f16)v; }
};

template <>
struct Store<bf16> {
    using C = float;
    __host__ __device__ static C widen(bf16 v) { return bf16_to_float(v); }
    __host__ __device__ static bf16 narrow(C v) { return float_to_bf16(v); }
};

// Source value -> compute type of storage T, rounded once to nearest even.
// For 16-bit T and an FP64 source the FP32 value is pinned in a register
// (empty asm) so that the compiler cannot fold FP64 -> FP32 -> FP16 into a
// single FP64 -> FP16 rounding: 16-bit state is always the rounding of the
// FP32 state.
template <typename T, typename S>
__device__ __forceinline__ typename Store<T>::C to_compute(S v)
{
    typename Store<T>::C c = (typename Store<T>::C)v;
    if constexpr (sizeof(T) == 2 && sizeof(S) == 8)
        __asm__ volatile("" : "+v"(c));
    return c;
}

}  // namespace fdtd
