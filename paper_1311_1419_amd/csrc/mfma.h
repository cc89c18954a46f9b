// Vector types and bf16 conversions shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace csv {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef int intx16 __attribute__((ext_vector_type(16)));

// bf16 bit pattern of a small integer (|v| <= 256): exact, the low half of
// its float encoding is zero.
__device__ inline uint16_t int_to_bf16_exact(int v) {
    return (uint16_t)(__float_as_uint((float)v) >> 16);
}

// Eight int8 values (|v| <= 32) widened exactly to bf16.
__device__ inline bf16x8 int8x8_to_bf16x8(uint2 w) {
    u16x8 o;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        o[i] = int_to_bf16_exact((int)(int8_t)((w.x >> (8 * i)) & 0xff));
        o[4 + i] = int_to_bf16_exact((int)(int8_t)((w.y >> (8 * i)) & 0xff));
    }
    return __builtin_bit_cast(bf16x8, o);
}

// float -> bf16 bits, round to nearest even (finite inputs).
__device__ __host__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace csv
