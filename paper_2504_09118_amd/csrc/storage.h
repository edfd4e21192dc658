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

// Round to nearest, ties to even; NaN stays a quiet NaN. On the device this is
// gfx950's conversion instruction (nearest even under the default rounding mode,
// FP32 denormals kept); the host form rounds the bits.
__host__ __device__ inline bf16 float_to_bf16(float f)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const __bf16 h = (__bf16)f;
    bf16 r;
    __builtin_memcpy(&r.u, &h, 2);
    return r;
#else
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
#endif
}

// Two FP32 values rounded to nearest even and packed as 16-bit values, a in the
// low half: one packed conversion instruction on gfx950 (v_cvt_pk_f16_f32,
// v_cvt_pk_bf16_f32).
typedef float pk_f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 pk_f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 pk_bf16x2 __attribute__((ext_vector_type(2)));

__device__ inline unsigned pack2_f16(float a, float b)
{
    const pk_f16x2 h = __builtin_convertvector((pk_f32x2){a, b}, pk_f16x2);
    unsigned u;
    __builtin_memcpy(&u, &h, 4);
    return u;
}

__device__ inline unsigned pack2_bf16(float a, float b)
{
    const pk_bf16x2 h = __builtin_convertvector((pk_f32x2){a, b}, pk_bf16x2);
    unsigned u;
    __builtin_memcpy(&u, &h, 4);
    return u;
}

// Compensated 16-bit storage: the 16-bit value (array of these) plus its rounding
// residual, an int8 in units of 1/256 of the 16-bit ulp, kept in a record with
// the residuals of the node's other two E (or H) components (kRecBytes below).
// Decoding is exact in FP32.
struct f16c {
    _Float16 h;
};
struct bf16c {
    unsigned short u;
};

template <typename S>
struct Store;

template <>
struct Store<float> {
    using C = float;
    static constexpr bool comp = false;
    __host__ __device__ static C widen(float v) { return v; }
    __host__ __device__ static float narrow(C v) { return v; }
};

template <>
struct Store<double> {
    using C = double;
    static constexpr bool comp = false;
    __host__ __device__ static C widen(double v) { return v; }
    __host__ __device__ static double narrow(C v) { return v; }
};

template <>
struct Store<f16> {
    using C = float;
    static constexpr bool comp = false;
    __host__ __device__ static C widen(f16 v) { return (float)v; }
    __host__ __device__ static f16 narrow(C v) { return (f16)v; }
    __device__ static unsigned pack2(C a, C b) { return pack2_f16(a, b); }
};

template <>
struct Store<bf16> {
    using C = float;
    static constexpr bool comp = false;
    __host__ __device__ static C widen(bf16 v) { return bf16_to_float(v); }
    __host__ __device__ static bf16 narrow(C v) { return float_to_bf16(v); }
    __device__ static unsigned pack2(C a, C b) { return pack2_bf16(a, b); }
};

__host__ __device__ inline unsigned f32_bits(float f)
{
    union {
        unsigned u;
        float f;
    } x;
    x.f = f;
    return x.u;
}

__host__ __device__ inline float bits_f32(unsigned u)
{
    union {
        unsigned u;
        float f;
    } x;
    x.u = u;
    return x.f;
}

// Compensated encoding of an FP32 value x: hi = x rounded to the 16-bit type
// (nearest even), r = x - hi (exact), residual q = rint(r / s) clamped to
// [-127, 127] with s = ulp(hi) / 256, a power of two taken from hi's exponent
// field e as 2^(max(e, e_min) - bias - mantissa_bits - 8). Decoding hi + q s is
// exact in FP32; the stored value is within s / 2 of x (ulp/512, 2^-20
// relative for FP16, 2^-17 for BF16).
__host__ __device__ inline float comp_scale_f16(unsigned short hbits)
{
    int e = (hbits >> 10) & 0x1f;
    e = e < 1 ? 1 : e;
    return bits_f32((unsigned)(e - 15 - 10 - 8 + 127) << 23);
}

__host__ __device__ inline float comp_scale_bf16(unsigned short hbits)
{
    int e = (hbits >> 7) & 0xff;
    e = e < 16 ? 16 : e;  // keeps the scale a normal FP32 number
    return bits_f32((unsigned)(e - 127 - 7 - 8 + 127) << 23);
}

// 1 / s for the encoder: also a power of two in the normal range (2^2..2^32 for FP16,
// 2^-113..2^126 for BF16), so r * (1/s) is the same correctly rounded value as r / s
// without a division sequence.
__host__ __device__ inline float comp_inv_scale_f16(unsigned short hbits)
{
    int e = (hbits >> 10) & 0x1f;
    e = e < 1 ? 1 : e;
    return bits_f32((unsigned)(15 + 10 + 8 - e + 127) << 23);
}

__host__ __device__ inline float comp_inv_scale_bf16(unsigned short hbits)
{
    int e = (hbits >> 7) & 0xff;
    e = e < 16 ? 16 : e;
    return bits_f32((unsigned)(127 + 7 + 8 - e + 127) << 23);
}

// The residual from the exact difference d = x - hi.
__host__ __device__ inline signed char comp_residual_d(float d, float inv_scale)
{
    const float q = __builtin_fminf(__builtin_fmaxf(__builtin_rintf(d * inv_scale), -127.0f), 127.0f);
    return (signed char)(int)q;
}

__host__ __device__ inline signed char comp_residual(float x, float hi, float inv_scale)
{
    // exact scaling by a power of two; |q| <= 128 for a finite x, so the clamp only folds
    // the half-ulp case 128 onto 127 (a NaN x gives hi = NaN, whatever q holds)
    const float q = __builtin_fminf(__builtin_fmaxf(__builtin_rintf((x - hi) * inv_scale), -127.0f), 127.0f);
    return (signed char)(int)q;
}

// Pair forms of the compensated codec for the sweeps: the same values as dec / enc on each
// element, with the two exponent fields handled by one packed 16-bit operation each
// (v_pk_* integer forms) instead of two scalar ones.
typedef unsigned short pk_u16x2 __attribute__((ext_vector_type(2)));

// Exponent fields of two 16-bit values (u: a in the low half) moved to the low bits,
// e = (u >> sh) & mask per half.
__device__ inline pk_u16x2 pair_exp(unsigned u, int sh, unsigned short mask)
{
    pk_u16x2 h;
    __builtin_memcpy(&h, &u, 4);
    return (h >> (pk_u16x2)(unsigned short)sh) & (pk_u16x2)mask;
}

// Signed byte 0 / byte 1 of q as FP32, each one conversion reading its byte directly.
__device__ inline float sbyte0_f32(unsigned q)
{
    float r;
    __asm__("v_cvt_f32_i32_sdwa %0, sext(%1) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_0"
            : "=v"(r)
            : "v"(q));
    return r;
}

__device__ inline float sbyte1_f32(unsigned q)
{
    float r;
    __asm__("v_cvt_f32_i32_sdwa %0, sext(%1) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_1"
            : "=v"(r)
            : "v"(q));
    return r;
}

__device__ inline float sbyte2_f32(unsigned q)
{
    float r;
    __asm__("v_cvt_f32_i32_sdwa %0, sext(%1) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_2"
            : "=v"(r)
            : "v"(q));
    return r;
}

// Signed byte B (0..2) of a word as FP32.
template <int B>
__device__ inline float sbyte_f32(unsigned q)
{
    if constexpr (B == 0)
        return sbyte0_f32(q);
    else if constexpr (B == 1)
        return sbyte1_f32(q);
    else
        return sbyte2_f32(q);
}

// FP32 powers of two whose exponent fields are the two halves of f (each < 256).
__device__ inline void pair_pow2(pk_u16x2 f, float &lo, float &hi)
{
    unsigned u;
    __builtin_memcpy(&u, &f, 4);
    lo = bits_f32(u << 23);                  // the high half shifts out
    hi = bits_f32((u >> 16) << 23);
}

template <>
struct Store<f16c> {
    using C = float;
    static constexpr bool comp = true;
    __host__ __device__ static unsigned short bits(f16c v)
    {
        unsigned short u;
        __builtin_memcpy(&u, &v, 2);
        return u;
    }
    __host__ __device__ static C dec(f16c hi, signed char q)
    {
        return (float)hi.h + (float)q * comp_scale_f16(bits(hi));
    }
    __host__ __device__ static void enc(C x, f16c &hi, signed char &q)
    {
        hi.h = (_Float16)x;
        q = comp_residual(x, (float)hi.h, comp_inv_scale_f16(bits(hi)));
    }
    // two values: the packed 16-bit pair (a low) and the packed residual bytes
    __device__ static void enc2(C a, C b, unsigned &hh, unsigned short &qq)
    {
        hh = pack2_f16(a, b);
        const unsigned short ua = (unsigned short)(hh & 0xffffu), ub = (unsigned short)(hh >> 16);
        _Float16 ha, hb;
        __builtin_memcpy(&ha, &ua, 2);
        __builtin_memcpy(&hb, &ub, 2);
        // 1/s = 2^(33 - max(e, 1)): exponent field 160 - max(e, 1)
        const pk_u16x2 e = __builtin_elementwise_max(pair_exp(hh, 10, 0x1f), (pk_u16x2)(unsigned short)1);
        float ia, ib;
        pair_pow2((pk_u16x2)(unsigned short)160 - e, ia, ib);
        // x - hi is exact in FP32
        const signed char qa = comp_residual_d(a - (float)ha, ia);
        const signed char qb = comp_residual_d(b - (float)hb, ib);
        qq = (unsigned short)((unsigned char)qa | ((unsigned)(unsigned char)qb << 8));
    }
    // two values from the packed pair u (a low) and the packed residual bytes q
    __device__ static void dec2(unsigned u, unsigned q, float &a, float &b)
    {
        // s = 2^(max(e, 1) - 33): exponent field max(e, 1) + 94
        const pk_u16x2 e = __builtin_elementwise_max(pair_exp(u, 10, 0x1f), (pk_u16x2)(unsigned short)1);
        float sa, sb;
        pair_pow2(e + (pk_u16x2)(unsigned short)94, sa, sb);
        const unsigned short ua = (unsigned short)(u & 0xffffu), ub = (unsigned short)(u >> 16);
        _Float16 ha, hb;
        __builtin_memcpy(&ha, &ua, 2);
        __builtin_memcpy(&hb, &ub, 2);
        a = (float)ha + sbyte0_f32(q) * sa;
        b = (float)hb + sbyte1_f32(q) * sb;
    }
    // the same from the residual records of the two cells (w0: cell a, w1: cell b), component B
    template <int B>
    __device__ static void dec2r(unsigned u, unsigned w0, unsigned w1, float &a, float &b)
    {
        const pk_u16x2 e = __builtin_elementwise_max(pair_exp(u, 10, 0x1f), (pk_u16x2)(unsigned short)1);
        float sa, sb;
        pair_pow2(e + (pk_u16x2)(unsigned short)94, sa, sb);
        const unsigned short ua = (unsigned short)(u & 0xffffu), ub = (unsigned short)(u >> 16);
        _Float16 ha, hb;
        __builtin_memcpy(&ha, &ua, 2);
        __builtin_memcpy(&hb, &ub, 2);
        a = (float)ha + sbyte_f32<B>(w0) * sa;
        b = (float)hb + sbyte_f32<B>(w1) * sb;
    }
};

template <>
struct Store<bf16c> {
    using C = float;
    static constexpr bool comp = true;
    __host__ __device__ static C dec(bf16c hi, signed char q)
    {
        return bf16_to_float(bf16{hi.u}) + (float)q * comp_scale_bf16(hi.u);
    }
    __host__ __device__ static void enc(C x, bf16c &hi, signed char &q)
    {
        hi.u = float_to_bf16(x).u;
        q = comp_residual(x, bf16_to_float(bf16{hi.u}), comp_inv_scale_bf16(hi.u));
    }
    __device__ static void enc2(C a, C b, unsigned &hh, unsigned short &qq)
    {
        hh = pack2_bf16(a, b);
        // 1/s = 2^(142 - max(e, 16)): exponent field 269 - max(e, 16), over 255 for e < 14,
        // so the packed form takes 269 - max(e, 16) in 16 bits (at most 253)
        const pk_u16x2 e = __builtin_elementwise_max(pair_exp(hh, 7, 0xff), (pk_u16x2)(unsigned short)16);
        float ia, ib;
        pair_pow2((pk_u16x2)(unsigned short)269 - e, ia, ib);
        const signed char qa = comp_residual(a, bits_f32(hh << 16), ia);
        const signed char qb = comp_residual(b, bits_f32(hh & 0xffff0000u), ib);
        qq = (unsigned short)((unsigned char)qa | ((unsigned)(unsigned char)qb << 8));
    }
    __device__ static void dec2(unsigned u, unsigned q, float &a, float &b)
    {
        // s = 2^(max(e, 16) - 142): exponent field max(e, 16) - 15
        const pk_u16x2 e = __builtin_elementwise_max(pair_exp(u, 7, 0xff), (pk_u16x2)(unsigned short)16);
        float sa, sb;
        pair_pow2(e - (pk_u16x2)(unsigned short)15, sa, sb);
        a = bits_f32(u << 16) + sbyte0_f32(q) * sa;
        b = bits_f32(u & 0xffff0000u) + sbyte1_f32(q) * sb;
    }
    template <int B>
    __device__ static void dec2r(unsigned u, unsigned w0, unsigned w1, float &a, float &b)
    {
        const pk_u16x2 e = __builtin_elementwise_max(pair_exp(u, 7, 0xff), (pk_u16x2)(unsigned short)16);
        float sa, sb;
        pair_pow2(e - (pk_u16x2)(unsigned short)15, sa, sb);
        a = bits_f32(u << 16) + sbyte_f32<B>(w0) * sa;
        b = bits_f32(u & 0xffff0000u) + sbyte_f32<B>(w1) * sb;
    }
};

// Compensated storage keeps the residuals of the three E (or H) components of a node
// together in one 4-byte record (byte c: component c, byte 3 zero), so that a sweep
// reads a lane's residuals with one load per group instead of one per component.
constexpr int kRecBytes = 4;

// Element access through the storage rules. lo: byte distance from a compensated
// box's element 0 to the byte of its component in the residual record of element 0
// (records kRecBytes apart; unused for the plain types).
template <typename T>
__host__ __device__ inline typename Store<T>::C get_elem(const T *a, long long lo, long long o)
{
    if constexpr (Store<T>::comp)
        return Store<T>::dec(a[o], ((const signed char *)a + lo)[kRecBytes * o]);
    else
        return Store<T>::widen(a[o]);
}

template <typename T>
__host__ __device__ inline void put_elem(T *a, long long lo, long long o, typename Store<T>::C v)
{
    if constexpr (Store<T>::comp) {
        T h;
        signed char q;
        Store<T>::enc(v, h, q);
        a[o] = h;
        ((signed char *)a + lo)[kRecBytes * o] = q;
    } else {
        a[o] = Store<T>::narrow(v);
    }
}

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
