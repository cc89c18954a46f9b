// Device Philox4x64-10 shared by the measurement-matrix kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace csv {

// ----------------------------------------------------------------- Philox
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128-bit products with the multipliers, the key advanced by the two
// Weyl increments before every round after the first.
__device__ inline void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3,
                                     uint64_t k0, uint64_t k1) {
    constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
    constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kW0;
            k1 += kW1;
        }
        const uint64_t lo0 = kM0 * c0, hi0 = __umul64hi(kM0, c0);
        const uint64_t lo1 = kM1 * c2, hi1 = __umul64hi(kM1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

}  // namespace csv
