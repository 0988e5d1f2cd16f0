// Low-precision number formats used by the patch network: bfloat16 (8
// exponent bits, 7 stored mantissa bits) and OCP FP8 E4M3FN (4 exponent bits,
// bias 7, 3 mantissa bits, largest finite 448, no infinities).  Conversions
// round to nearest, ties to even; the FP8 encoder saturates at +-448.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dnnmg {

__host__ __device__ __forceinline__ uint32_t f32_bits(float f) {
    union {
        float f;
        uint32_t u;
    } c;
    c.f = f;
    return c.u;
}

__host__ __device__ __forceinline__ float bits_f32(uint32_t u) {
    union {
        float f;
        uint32_t u;
    } c;
    c.u = u;
    return c.f;
}

// float -> bfloat16 bits: add half an ulp of the 16-bit result (minus one
// when the kept part is even) and truncate.
__host__ __device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = f32_bits(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u); // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ __forceinline__ float bf16_to_f32(uint16_t h) { return bits_f32((uint32_t)h << 16); }

__host__ __device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    return (uint32_t)f32_to_bf16(lo) | ((uint32_t)f32_to_bf16(hi) << 16);
}

// The same conversions with gfx950's packed f32 -> bf16 instruction (round to
// nearest even; bit for bit equal to f32_to_bf16 for every non-NaN input, and
// NaN stays NaN), for device code.
typedef __bf16 dnnmg_bf16x2 __attribute__((ext_vector_type(2)));
typedef float dnnmg_f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2_hw(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((dnnmg_f32x2){lo, hi}, dnnmg_bf16x2));
}
__device__ __forceinline__ uint16_t f32_to_bf16_hw(float f) { return (uint16_t)pack_bf16x2_hw(f, 0.0f); }

// float -> E4M3FN bits.  Normal range 2^-6 .. 448 keeps 3 mantissa bits;
// below 2^-6 the spacing is 2^-9 (subnormals).
__host__ __device__ __forceinline__ uint8_t f32_to_e4m3(float f) {
    uint32_t u = f32_bits(f);
    uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
    uint32_t a = u & 0x7fffffffu;
    if (a > 0x7f800000u) return 0x7f; // NaN
    float af = bits_f32(a);
    if (af >= 448.0f) return sign | 0x7e; // saturate
    if (af < 0.015625f) {                 // subnormal: m * 2^-9, m = 0..8
        float s = af * 512.0f;            // exact scaling
        // round half to even on a value < 8
        float fl = floorf(s);
        float fr = s - fl;
        uint32_t mi = (uint32_t)fl;
        if (fr > 0.5f || (fr == 0.5f && (mi & 1u))) ++mi;
        return sign | (uint8_t)mi; // mi == 8 encodes 2^-6 (exponent field 1)
    }
    // normal: round the 23-bit mantissa to 3 bits
    a += 0x7ffffu + ((a >> 20) & 1u);
    int e = (int)(a >> 23) - 127; // -6 .. 8
    uint32_t m3 = (a >> 20) & 7u;
    uint32_t code = ((uint32_t)(e + 7) << 3) | m3;
    if (code > 0x7eu) code = 0x7eu;
    return sign | (uint8_t)code;
}

__host__ __device__ __forceinline__ float e4m3_to_f32(uint8_t c) {
    uint32_t e = (c >> 3) & 15u, m = c & 7u;
    float v;
    if (e == 15u && m == 7u) return bits_f32(0x7fc00000u);
    if (e == 0u) v = (float)m * (1.0f / 512.0f);
    else v = bits_f32(((e - 7u + 127u) << 23) | (m << 20));
    return (c & 0x80u) ? -v : v;
}

} // namespace dnnmg
