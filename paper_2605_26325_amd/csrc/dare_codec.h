// Storage codecs of the directional grid: FP32 / BF16 / FP16 / FP8 (OCP e4m3fn).
//
// Per voxel the grid stores a mean intensity a = fl32(S) / fl32(C) and a
// sample count C.  The 16-bit forms store q = round(fl32(fl32(a - 127.5) *
// fl32(1 / 127.5))) so that the value range [0, 255] maps onto [-1, 1], and
// read back a = fl32(fl32(q * 127.5) + 127.5).  FP8 stores q = round(fl32(
// fl32(a - 127.5) / s)) with one FP32 scale s per (bin, brick) and the count
// as round(fl32(C / t)) with a second per-brick scale t.  Rounding is to
// nearest, ties to even; e4m3 results beyond 448 saturate to 448.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "../../include/dare.h"

// Stored values decode as fl32(fl32(q * s) + 127.5): no fused multiply-add.
#pragma clang fp contract(off)

namespace dare {

__device__ __forceinline__ uint32_t f32_to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ __forceinline__ float bf16_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

__device__ __forceinline__ uint32_t f32_to_f16_rne(float x) {
    return (uint32_t)__half_as_ushort(__float2half_rn(x));
}

__device__ __forceinline__ float f16_to_f32(uint32_t hbits) {
    return __half2float(__ushort_as_half((unsigned short)hbits));
}

// float -> OCP e4m3fn code, round to nearest even, saturating at 448.
__device__ __forceinline__ uint32_t f32_to_e4m3_rne(float x) {
    uint32_t u = __float_as_uint(x);
    uint32_t sign = (u >> 31) << 7;
    float ax = fabsf(x);
    uint32_t code;
    if (!(ax < 464.0f)) {                         // at or beyond the rounding edge of 448
        code = 0x7Eu;                             // (also maps NaN to 448; inputs are finite)
    } else if (ax < 0.015625f) {                  // below the smallest normal 2^-6
        code = (uint32_t)__builtin_rintf(ax * 512.0f);   // multiples of 2^-9; 8 becomes 2^-6
    } else {
        uint32_t au = __float_as_uint(ax);
        int e = (int)((au >> 23) & 0xFFu) - 127;  // -6 .. 8
        uint32_t mant = au & 0x7FFFFFu;
        uint32_t r = mant >> 20;
        uint32_t rem = mant & 0xFFFFFu;
        if (rem > 0x80000u || (rem == 0x80000u && (r & 1u))) ++r;
        if (r == 8u) { r = 0u; ++e; }
        if (e > 8 || (e == 8 && r == 7u)) code = 0x7Eu;
        else code = ((uint32_t)(e + 7) << 3) | r;
    }
    return sign | code;
}

__device__ __forceinline__ float e4m3_to_f32(uint32_t c) {
    uint32_t e = (c >> 3) & 15u, m = c & 7u;
    float v = (e == 0u) ? (float)m * 0.001953125f                 // m * 2^-9, exact
                        : __uint_as_float(((e + 120u) << 23) | (m << 20));
    return (c & 0x80u) ? -v : v;
}

template <int DT> struct Pair;

template <> struct Pair<DARE_F32> {
    using T = float2;
    __device__ __forceinline__ static void decode(T p, float2, float& a, float& c) { a = p.x; c = p.y; }
};
template <> struct Pair<DARE_BF16> {
    using T = uint32_t;
    __device__ __forceinline__ static void decode(T p, float2, float& a, float& c) {
        float q = __uint_as_float(p << 16);
        a = q * 127.5f;
        a = a + 127.5f;
        c = __uint_as_float(p & 0xFFFF0000u);
    }
};
template <> struct Pair<DARE_F16> {
    using T = uint32_t;
    __device__ __forceinline__ static void decode(T p, float2, float& a, float& c) {
        float q = f16_to_f32(p & 0xFFFFu);
        a = q * 127.5f;
        a = a + 127.5f;
        c = f16_to_f32(p >> 16);
    }
};
template <> struct Pair<DARE_FP8_E4M3> {
    using T = uint16_t;
    __device__ __forceinline__ static void decode(T p, float2 s, float& a, float& c) {
        float q = e4m3_to_f32(p & 0xFFu);
        a = q * s.x;
        a = a + 127.5f;
        c = e4m3_to_f32(p >> 8) * s.y;
    }
};

}  // namespace dare
