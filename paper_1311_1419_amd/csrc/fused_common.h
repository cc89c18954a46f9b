// Device helpers shared by the fused BF16 recovery kernels (FISTA and TV):
// global-memory pointer types, the K order of the fragments, packing, the
// per-XCD tile queues and the forward product with its residual epilogue.
#pragma once

#include <type_traits>
#include "internal.h"
#include "mfma.h"

namespace csv {

// Pointers into global memory.  Tile descriptors are read from memory, so
// without the address space the compiler emits flat loads, which count on
// the LDS counter too and force a full wait before every LDS read.
typedef __attribute__((address_space(1))) const u16x8 gu16x8;
typedef __attribute__((address_space(1))) const float gfloat;
// Tables the kernel only reads, at addresses uniform over the workgroup
// (the momentum factors, the step constant): through the constant address
// space with a uniform address these become scalar loads, which the wave
// does not wait for before its next LDS access the way it waits for a
// flat load.
typedef __attribute__((address_space(4))) const float cfloat;
typedef __attribute__((address_space(4))) const double cdouble;
template <class T>
__device__ inline T* as_global(const void* p) {
    return (T*)(p);
}

// K index inside a 32-group carried by (K step s, lane half h, element e).
__host__ __device__ inline int kappa(int s, int h, int e) {
    return 16 * s + 8 * (e / 4) + 4 * h + (e % 4);
}

__device__ inline u16x8 pack_bf16(const floatx16& a, int s) {
    u16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = __builtin_bit_cast(uint16_t, (__bf16)a[8 * s + e]);
    return o;
}

__device__ inline int next_tile(const int* __restrict__ qoff, const int* __restrict__ queue,
                                int* __restrict__ counters) {
    const int x0 = blockIdx.x & 7;
    for (int d = 0; d < 8; ++d) {
        const int x = (x0 + d) & 7;
        const int len = qoff[x + 1] - qoff[x];
        if (len <= 0) continue;
        const int i = atomicAdd(&counters[x], 1);
        if (i < len) return queue[qoff[x] + i];
    }
    return -1;
}


// Forward product for this wave's NF output tiles (mt_i, fct), mt_i =
// (w + W i) / CT.  af holds the first kPF K steps on entry.  Loads the first
// kPA adjoint steps (rows rt0 + r / CT) into aa before returning.  With
// NL > 0 the last NL K steps of every tile come from the wave's LDS copy Al
// ([NF][NL][64] fragments) instead of global memory: after the global steps,
// or with ILV one after each of the first NL rounds of the global ring, so
// that the ring's loads stay in flight while they run.  The operator
// pointers (type PT) address global memory, or a copy of the whole operator
// in LDS.
template <int N, int MP, int CT, int NF, int AR, int W, int kPF, int kPA, int NL = 0,
          bool ILV = false, class PT = gu16x8, class PTA = PT>
__device__ inline void forward_tiles(u16x8 (&af)[kPF][NF], u16x8 (&aa)[kPA][AR],
                                     floatx16 (&acc)[NF], const PT* ffwd, const PTA* fadj,
                                     const u16x8* Vb, int w, int ln, int fct, int rt0,
                                     const u16x8* Al = nullptr) {
    constexpr int KSF = N / 16, KSA = MP / 16, KSG = KSF - NL;
    static_assert(NL >= 0 && KSG >= kPF && KSG % kPF == 0, "LDS steps must leave whole rings");
    static_assert(kPA <= kPF, "the adjoint head is loaded during the last kPF forward steps");
    static_assert(!ILV || (KSG - kPF) / kPF >= NL, "too few ring rounds to interleave");
    auto lds_step = [&](int j) {
        const int ks = KSG + j;
        const bf16x8 b = __builtin_bit_cast(bf16x8, Vb[(ks * CT + fct) * 64 + ln]);
#pragma unroll
        for (int i = 0; i < NF; ++i)
            acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, Al[(i * NL + j) * 64 + ln]), b, acc[i], 0, 0, 0);
    };
#pragma unroll
    for (int i = 0; i < NF; ++i) acc[i] = floatx16{};
    if constexpr (KSG <= 16 && NL == 0 && std::is_same_v<PT, u16x8>) {
        // short product on an LDS-resident operator (n = 256): fully
        // unrolled, so the first step takes a zero accumulator operand and
        // every fragment address is an immediate offset
#pragma unroll
        for (int ks0 = 0; ks0 < KSG - kPF; ks0 += kPF) {
#pragma unroll
            for (int j = 0; j < kPF; ++j) {
                const int ks = ks0 + j;
                const bf16x8 b = __builtin_bit_cast(bf16x8, Vb[(ks * CT + fct) * 64 + ln]);
#pragma unroll
                for (int i = 0; i < NF; ++i) {
                    acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, af[j][i]), b, acc[i], 0, 0, 0);
                    const int mt = (w + W * i) / CT;
                    af[j][i] = ffwd[((size_t)mt * KSF + ks + kPF) * 64 + ln];
                }
            }
        }
    } else {
#pragma unroll 1
        for (int ks0 = 0; ks0 < KSG - kPF; ks0 += kPF) {
#pragma unroll
            for (int j = 0; j < kPF; ++j) {
                const int ks = ks0 + j;
                const bf16x8 b = __builtin_bit_cast(bf16x8, Vb[(ks * CT + fct) * 64 + ln]);
#pragma unroll
                for (int i = 0; i < NF; ++i) {
                    acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, af[j][i]), b, acc[i], 0, 0, 0);
                    const int mt = (w + W * i) / CT;
                    af[j][i] = ffwd[((size_t)mt * KSF + ks + kPF) * 64 + ln];
                }
            }
            if constexpr (ILV && NL > 0) {
                if (ks0 / kPF < NL) lds_step(ks0 / kPF);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kPF; ++j) {   // last kPF global steps: no further forward loads
        const int ks = KSG - kPF + j;
        const bf16x8 b = __builtin_bit_cast(bf16x8, Vb[(ks * CT + fct) * 64 + ln]);
#pragma unroll
        for (int i = 0; i < NF; ++i)
            acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, af[j][i]), b,
                                                             acc[i], 0, 0, 0);
        if (j < kPA) {
#pragma unroll
            for (int r = 0; r < AR; ++r)
                aa[j][r] = fadj[((size_t)(rt0 + r / CT) * KSA + j) * 64 + ln];
        }
    }
    if constexpr (!ILV) {
#pragma unroll
        for (int j = 0; j < NL; ++j) lds_step(j);   // LDS-resident steps
    }
}

template <int N, int MP, int CT, int NF, int W, int kPF, class PT = gu16x8>
__device__ inline void load_fwd_head(u16x8 (&af)[kPF][NF], const PT* ffwd, int w, int ln) {
    constexpr int KSF = N / 16;
#pragma unroll
    for (int p = 0; p < kPF; ++p)
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const int mt = (w + W * i) / CT;
            af[p][i] = ffwd[((size_t)mt * KSF + p) * 64 + ln];
        }
}

// R = P - y for one forward tile, written to LDS as bf16 (y from registers
// or from global memory).  NEG: R' = (y - P) * scale instead, so that an
// adjoint accumulator started at v ends at v - A^T (P - y) scale; with y in
// registers it is held as y * scale and R' = y * scale - P * scale.
template <int MP, int CT, bool YREG, bool NEG = false>
__device__ inline void store_residual(const floatx16& acc, const floatx16& yv, const gfloat* yg,
                                      int nblk, int mt, int fct, int ln, u16x8* Rb,
                                      float scale = 1.f) {
    const int h = ln >> 5, b = fct * 32 + (ln & 31);
    floatx16 yy = {};
    if constexpr (YREG) {
        yy = yv;
    } else if (b < nblk) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const gfloat* yp = yg + (size_t)b * MP + mt * 32 + 8 * q + 4 * h;
            yy[4 * q] = yp[0];
            yy[4 * q + 1] = yp[1];
            yy[4 * q + 2] = yp[2];
            yy[4 * q + 3] = yp[3];
        }
    }
    floatx16 rr;
#pragma unroll
    for (int r = 0; r < 16; ++r)
        rr[r] = !NEG ? acc[r] - yy[r] : YREG ? fmaf(-acc[r], scale, yy[r]) : (yy[r] - acc[r]) * scale;
    Rb[((2 * mt) * CT + fct) * 64 + ln] = pack_bf16(rr, 0);
    Rb[((2 * mt + 1) * CT + fct) * 64 + ln] = pack_bf16(rr, 1);
}

}  // namespace csv
