// Fused BF16 recovery: all T FISTA iterations of a tile of 32*CT blocks run
// inside one workgroup, iterates on chip, both products on MFMA.
//
// Problem per block (eq. (1) read as a LASSO in the 2-D DCT basis):
//   min_s 1/2 ||A s - y||^2 + lam ||s||_1,   A = Phi Psi (M x n)
// FISTA with constant step 1/L (Beck and Teboulle 2009):
//   u = v - A^T (A v - y) / L;  s_k = soft(u, lam / L);
//   v = s_k + beta_k (s_k - s_{k-1}).
//
// Layout.  A workgroup is eight waves (two per SIMD); wave w owns
// coefficient rows [w n/8, (w+1) n/8) of every block of the tile and keeps s_{k-1} and v in
// FP32 registers, in the 32x32 MFMA accumulator layout (lane l, register r:
// row 8(r/4) + 4(l/32) + r%4 of a 32-row group, column l%32).  Per
// iteration:
//   forward  P = A V  (M x 32CT, K = n): output tiles split over the waves by
//            M rows; V comes from LDS as bf16 B fragments; A streams from
//            global memory (L2) as bf16 A fragments;  R' = (y - P) / L
//            (FP32, y read from L2) is written back to LDS as bf16;
//   adjoint  u = V + A^T R'  (n x 32CT, K = M): each wave computes its own
//            rows, its accumulators started at v, R' from LDS, A^T streamed
//            as bf16 fragments, so the product ends at the gradient step
//            u = v - A^T (A v - y) / L; the threshold and momentum update
//            runs on the accumulators in registers and the new V is written
//            to LDS as bf16.
// A 32-row accumulator tile feeds the next product's K dimension without a
// shuffle: in K step s of a 32x32x16 MFMA, lane half h, element e carries
// row kappa_s(h, e) = 16 s + 8 (e / 4) + 4 h + e % 4 of the group, which is
// register 8 s + e of the accumulator.  The operator fragments are stored
// with that same K order, so the products are exact permutations of the
// plain sums.
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "fused_common.h"

namespace csv {


// frag_fwd[mt][ks][lane][e] = A[mt*32 + lane%32][32*(ks/2) + kappa(ks%2, lane/32, e)]
// frag_adj[nt][ks][lane][e] = A[32*(ks/2) + kappa(ks%2, lane/32, e)][nt*32 + lane%32]
__global__ void frag_layout_kernel(const float* __restrict__ a32, int n, int Mp,
                                   uint16_t* __restrict__ fwd, uint16_t* __restrict__ adj) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)Mp * n;
    if (idx >= total) return;
    const int e = (int)(idx & 7), lane = (int)((idx >> 3) & 63);
    const size_t frag = idx >> 9;
    const int h = lane >> 5, i = lane & 31;
    {   // forward: fragments ordered [mt][ks], ks over n/16
        const int ks = (int)(frag % (n / 16)), mt = (int)(frag / (n / 16));
        const int row = mt * 32 + i, col = 32 * (ks / 2) + kappa(ks % 2, h, e);
        fwd[idx] = f32_to_bf16_rne(a32[(size_t)row * n + col]);
    }
    {   // adjoint: fragments ordered [nt][ks], ks over Mp/16
        const int ks = (int)(frag % (Mp / 16)), nt = (int)(frag / (Mp / 16));
        const int row = 32 * (ks / 2) + kappa(ks % 2, h, e), col = nt * 32 + i;
        adj[idx] = f32_to_bf16_rne(a32[(size_t)row * n + col]);
    }
}

void launch_bf16_frag_layout(Operator* op, hipStream_t st) {
    const size_t total = (size_t)op->Mp * op->n;
    frag_layout_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st>>>(
        op->a32, op->n, op->Mp, op->frag_fwd, op->frag_adj);
    CSV_HIP(hipGetLastError());
    // Phi itself (pixel-domain products of the TV solver)
    frag_layout_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st>>>(
        op->phi32, op->n, op->Mp, op->phi_frag_fwd, op->phi_frag_adj);
    CSV_HIP(hipGetLastError());
}

// SPL: accumulator tiles per wave whose s_{k-1} lives in LDS rather than in
// registers (the registers go to deeper operator rings instead).  OCC
// workgroups share a CU, so a wave gets 512 / (W OCC / 4) registers.
// NL: the last NL forward K steps of each wave's operator rows are kept in
// LDS, copied when a tile's operator differs from the previous tile's, so
// that every iteration reads NL fewer fragments through the L1 return path
// (the kernel's bound at n = 1024).  NL < 0: -NL such steps, interleaved
// with the global ring rounds instead of run after them.  OPT bit 0: each
// wave keeps its y^ rows of the tile in registers for all T iterations
// instead of reading them from L2 in every residual epilogue.  OPT bit 1:
// both fragment layouts of the whole operator are copied to LDS when a
// tile's operator differs from the previous tile's, and every iteration
// reads them there instead of from L2 (small classes, where the operator
// fits beside V and R).  OPT bit 2: s and v in two register arrays that
// trade roles every iteration (implied by bits 0 and 1 together).  OPT bit
// 3: only the adjoint layout of the operator is copied to LDS, the forward
// one streams from L2 (classes where one layout fits beside V and R).
template <int N, int MP, int CT, int W, int kPF, int kPA, int SPL, int OCC, int NLS, int OPT = 0>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(W * OCC / 4)))
void fista_bf16_kernel(
    const FusedTile* __restrict__ tiles, const int* __restrict__ qoff,
    const int* __restrict__ queue, int* __restrict__ counters) {
    constexpr int RT = N / 32 / W;               // 32-row groups of n owned per wave
    constexpr int NG = RT * CT / 2;              // adjoint groups of two accumulator tiles
    constexpr int UT = RT * CT;                  // accumulator tiles (rt, ct), u = rt * CT + ct
    constexpr int SPR = UT - SPL;                // tiles whose s_{k-1} stays in registers
    static_assert(SPL >= 0 && SPL <= UT, "bad LDS state split");
    constexpr int AR = CT == 1 ? 2 : 1;          // distinct operator rows per group
    constexpr int TT = (MP / 32) * CT;           // forward output tiles
    constexpr int FT = (TT + W - 1) / W;         // forward tiles per wave (max)
    constexpr int KSF = N / 16, KSA = MP / 16;   // K steps of forward / adjoint
    constexpr bool YREG = (OPT & 1) != 0;        // else y^ is read from L2 in every epilogue
    constexpr bool OPL = (OPT & 2) != 0;         // operator resident in LDS
    constexpr bool OPA = (OPT & 8) != 0;         // adjoint layout alone resident in LDS
    static_assert(!(OPL && OPA), "the adjoint layout is part of an LDS-resident operator");
    constexpr bool PP = (YREG && OPL) || (OPT & 4) != 0;   // ping-pong state
    static_assert(!PP || SPL == 0, "ping-pong state keeps every tile in registers");
    static_assert(!(OPL && NLS != 0), "the LDS slice is part of an LDS-resident operator");
    constexpr int OFW = (MP / 32) * KSF * 64;   // u16x8 of the forward layout (OPL)
    constexpr int OFA = (N / 32) * KSA * 64;    // u16x8 of the adjoint layout (OPL)
    using PT = std::conditional_t<OPL, u16x8, gu16x8>;   // forward operator pointee type
    using PTA = std::conditional_t<OPL || OPA, u16x8, gu16x8>;   // adjoint's
    constexpr int NL = NLS < 0 ? -NLS : NLS;     // LDS-resident forward K steps
    constexpr bool ILV = NLS < 0;
    static_assert(RT * CT >= 2 && (RT * CT) % 2 == 0 && W % CT == 0, "unsupported class");
    static_assert(KSF % kPF == 0 && KSA % kPA == 0 && KSF >= kPF && KSA >= kPA,
                  "ring depth must divide the K steps");
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    u16x8* Vb = reinterpret_cast<u16x8*>(lds);                            // [KSF][CT][64]
    u16x8* Rb = reinterpret_cast<u16x8*>(lds + (size_t)KSF * CT * 1024);  // [KSA][CT][64]
    float4* Sl = reinterpret_cast<float4*>(lds + (size_t)(KSF + KSA) * CT * 1024);
    // Sl: [W][SPL][4][64] float4, lane l's 16 values of a tile at q * 64 + l
    u16x8* Al = reinterpret_cast<u16x8*>(lds + (size_t)(KSF + KSA) * CT * 1024 +
                                         (size_t)W * SPL * 4096);
    // Al: [W][FT][NL][64], forward fragments (mt_i, KSF - NL + j) of wave w
    u16x8* Ol = Al + (size_t)W * FT * NL * 64;
    // Ol (OPL): [forward layout OFW][adjoint layout OFA], the global order;
    // (OPA): [adjoint layout OFA]
    static_assert(NL == 0 || KSF - NL >= kPF, "LDS steps leave no global ring");
    __shared__ int s_tile;

    const int tid = threadIdx.x, w = tid >> 6, ln = tid & 63, h = ln >> 5, col = ln & 31;
    const int fct = w % CT;                      // column tile of this wave's forward tiles
    const int nft = (TT - w + W - 1) / W;        // forward tiles of this wave: FT, FT-1 or 0
    const void* al_src = nullptr;                // operator whose fragments Al holds
    const void* ol_src = nullptr;                // operator that Ol holds (OPL)

    for (;;) {
        if (tid == 0) s_tile = next_tile(qoff, queue, counters);
        __syncthreads();
        // uniform: the descriptor and the tables it points to are then
        // read with scalar loads
        const int t_id = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (t_id < 0) break;
        const FusedTile tl = tiles[t_id];
        const PT* ffwd;
        const PTA* fadj;
        if constexpr (OPA) {
            // as OPL below, the adjoint layout only
            if (tl.frag_adj != ol_src) {
                const gu16x8* ga = as_global<const gu16x8>(tl.frag_adj);
                for (int i = tid; i < OFA; i += 64 * W) Ol[i] = ga[i];
                ol_src = tl.frag_adj;
                __syncthreads();
            }
            ffwd = as_global<const gu16x8>(tl.frag_fwd);
            fadj = Ol;
        } else if constexpr (OPL) {
            // every wave is past the previous tile (barriers above): copy the
            // new tile's operator once, then wait for the whole copy
            if (tl.frag_fwd != ol_src) {
                const gu16x8* gf = as_global<const gu16x8>(tl.frag_fwd);
                const gu16x8* ga = as_global<const gu16x8>(tl.frag_adj);
                for (int i = tid; i < OFW; i += 64 * W) Ol[i] = gf[i];
                for (int i = tid; i < OFA; i += 64 * W) Ol[OFW + i] = ga[i];
                ol_src = tl.frag_fwd;
                __syncthreads();
            }
            ffwd = Ol;
            fadj = Ol + OFW;
        } else {
            ffwd = as_global<const gu16x8>(tl.frag_fwd);
            fadj = as_global<const gu16x8>(tl.frag_adj);
        }
        const gfloat* yg = as_global<const gfloat>(tl.y);
        const float inv_l = (float)(1.0 / as_global<cdouble>(tl.lip)[0]);
        const int T = tl.T;
        const cfloat* __restrict__ beta = as_global<cfloat>(tl.beta);
        const gfloat* __restrict__ lamg = as_global<gfloat>(tl.lam);
        if constexpr (NL > 0) {
            // each lane reads back only what it wrote itself: no barrier
            if (nft == FT && tl.frag_fwd != al_src) {
#pragma unroll
                for (int i = 0; i < FT; ++i)
#pragma unroll
                    for (int j = 0; j < NL; ++j)
                        Al[((w * FT + i) * NL + j) * 64 + ln] =
                            ffwd[((size_t)((w + W * i) / CT) * KSF + KSF - NL + j) * 64 + ln];
                al_src = tl.frag_fwd;
            }
        }

        float tau[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int b = ct * 32 + col;
            tau[ct] = b < tl.nblk ? lamg[b] * inv_l : 0.f;
        }
        floatx16 yv[YREG ? FT : 1];
        if constexpr (YREG) {
#pragma unroll
            for (int i = 0; i < FT; ++i) {
                const int t = w + W * i;
                const int mt = t / CT;
                const int b = fct * 32 + col;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int m = mt * 32 + 8 * (r / 4) + 4 * h + (r % 4);
                    // held as y^ / L: the residual epilogue is then one FMA
                    yv[i][r] = (t < TT && b < tl.nblk) ? yg[(size_t)b * MP + m] * inv_l : 0.f;
                }
            }
        }
        // PP: vv and pp swap roles every iteration (see the threshold below)
        floatx16 sp[(SPR > 0 && !PP) ? SPR : 1], vv[RT][CT], pp[RT][CT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int u = rt * CT + ct;
                if (!PP && u < SPR) sp[u] = floatx16{};
                if constexpr (PP) pp[rt][ct] = floatx16{};
                vv[rt][ct] = floatx16{};
                const int g = w * RT + rt;
                const u16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
                Vb[((2 * g) * CT + ct) * 64 + ln] = z;
                Vb[((2 * g + 1) * CT + ct) * 64 + ln] = z;
            }
#pragma unroll
        for (int t = 0; t < SPL; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                Sl[((w * SPL + t) * 4 + q) * 64 + ln] = make_float4(0.f, 0.f, 0.f, 0.f);
        u16x8 af[kPF][FT];
        u16x8 aa[kPA][AR];
        if (nft == FT) load_fwd_head<N, MP, CT, FT, W, kPF>(af, ffwd, w, ln);
        __syncthreads();

        // Iterations in pairs (PP) or one at a time.  X: the accumulators, v
        // on entry; Y (PP only): p = -beta_k s_{k-1} on entry.  PP leaves v in
        // Y and the next p in X, so the arrays trade roles every iteration.
        constexpr int NP = PP ? 2 : 1;
        for (int k0 = 0; k0 < T; k0 += NP) {
#pragma unroll
          for (int par = 0; par < NP; ++par) {
            const int k = k0 + par;
            if (NP == 2 && k >= T) break;
            floatx16 (&X)[RT][CT] = par ? pp : vv;
            floatx16 (&Y)[RT][CT] = par ? vv : pp;
            // ---- forward: P = A V, R = P - y  (nft tiles for this wave)
            if (nft == FT) {
                floatx16 acc[FT];
                forward_tiles<N, MP, CT, FT, AR, W, kPF, kPA, NL, ILV>(af, aa, acc, ffwd, fadj, Vb, w, ln,
                                                                  fct, w * RT,
                                                                  Al + (size_t)w * FT * NL * 64);
#pragma unroll
                for (int i = 0; i < FT; ++i)
                    store_residual<MP, CT, YREG, true>(acc[i], yv[YREG ? i : 0], yg, tl.nblk,
                                                       (w + W * i) / CT, fct, ln, Rb, inv_l);
            } else {
                bool done = false;
                if constexpr (FT > 1) {
                    if (nft == FT - 1) {
                        u16x8 af2[kPF][FT - 1];
                        floatx16 acc[FT - 1];
                        load_fwd_head<N, MP, CT, FT - 1, W, kPF>(af2, ffwd, w, ln);
                        forward_tiles<N, MP, CT, FT - 1, AR, W, kPF, kPA>(af2, aa, acc, ffwd, fadj,
                                                                          Vb, w, ln, fct, w * RT);
#pragma unroll
                        for (int i = 0; i < FT - 1; ++i)
                            store_residual<MP, CT, YREG, true>(acc[i], yv[YREG ? i : 0], yg,
                                                               tl.nblk, (w + W * i) / CT, fct, ln,
                                                               Rb, inv_l);
                        done = true;
                    }
                }
                if (!done) {
#pragma unroll
                    for (int p = 0; p < kPA; ++p)
#pragma unroll
                        for (int r = 0; r < AR; ++r)
                            aa[p][r] = fadj[((size_t)(w * RT + r / CT) * KSA + p) * 64 + ln];
                }
            }
            __syncthreads();
            // ---- adjoint G = A^T R over the wave's RT x CT accumulator tiles,
            //      two at a time (items u = 2g, 2g+1 of the row-major (rt, ct)
            //      list); threshold and momentum on the accumulators; new V
            //      to LDS
            const float bk = beta[k];
            const float bk1 = 1.f + bk, nbk = -bk;
            // PP: p for the next iteration, -beta_{k+1} s_k; after the last
            // iteration X holds s_T itself
            const float nbn = PP ? (k + 1 < T ? -beta[k + 1] : 1.f) : 0.f;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                        const int rt0 = (2 * g) / CT, ct0 = (2 * g) % CT;
                const int rt1 = (2 * g + 1) / CT, ct1 = (2 * g + 1) % CT;
                // accumulated in place on v: with R' = (y - A v) / L the
                // product ends at u = v - A^T (A v - y) / L
                floatx16& ga0 = X[rt0][ct0];
                floatx16& ga1 = X[rt1][ct1];
#pragma unroll 1
                for (int ks0 = 0; ks0 < KSA - kPA; ks0 += kPA) {
#pragma unroll
                    for (int j = 0; j < kPA; ++j) {
                        const int ks = ks0 + j;
                        const bf16x8 b0 = __builtin_bit_cast(bf16x8, Rb[(ks * CT + ct0) * 64 + ln]);
                        const bf16x8 b1 =
                            ct1 == ct0 ? b0
                                       : __builtin_bit_cast(bf16x8, Rb[(ks * CT + ct1) * 64 + ln]);
                        const bf16x8 a0 = __builtin_bit_cast(bf16x8, aa[j][0]);
                        const bf16x8 a1 = AR == 2 ? __builtin_bit_cast(bf16x8, aa[j][AR - 1]) : a0;
                        ga0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, ga0, 0, 0, 0);
                        ga1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, ga1, 0, 0, 0);
#pragma unroll
                        for (int r = 0; r < AR; ++r)
                            aa[j][r] = fadj[((size_t)(w * RT + (2 * g + r) / CT) * KSA + ks + kPA) *
                                                64 + ln];
                    }
                }
#pragma unroll
                for (int j = 0; j < kPA; ++j) {   // last kPA steps: prefetch the next group's head
                    const int ks = KSA - kPA + j;
                    const bf16x8 b0 = __builtin_bit_cast(bf16x8, Rb[(ks * CT + ct0) * 64 + ln]);
                    const bf16x8 b1 =
                        ct1 == ct0 ? b0 : __builtin_bit_cast(bf16x8, Rb[(ks * CT + ct1) * 64 + ln]);
                    const bf16x8 a0 = __builtin_bit_cast(bf16x8, aa[j][0]);
                    const bf16x8 a1 = AR == 2 ? __builtin_bit_cast(bf16x8, aa[j][AR - 1]) : a0;
                    ga0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, ga0, 0, 0, 0);
                    ga1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, ga1, 0, 0, 0);
                    if (g + 1 < NG) {
#pragma unroll
                        for (int r = 0; r < AR; ++r)
                            aa[j][r] = fadj[((size_t)(w * RT + (2 * (g + 1) + r) / CT) * KSA + j) *
                                                64 + ln];
                    }
                }
                if (g == NG - 1 && nft == FT) load_fwd_head<N, MP, CT, FT, W, kPF>(af, ffwd, w, ln);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int rt = e ? rt1 : rt0, ct = e ? ct1 : ct0;
                    const int ut = 2 * g + e;
                    const int gg = w * RT + rt;
                    const float tc = tau[ct];
                    if constexpr (PP) {
                        // s_k = u - med3(u, -tau, tau); v = (1 + beta_k) s_k + p, where
                        // p = -beta_k s_{k-1} was formed by the previous iteration
                        // (the same two roundings as forming it here).  The two
                        // state arrays trade roles each iteration, so the four
                        // VALU operations write in place with no register moves
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const float u = X[rt][ct][r];
                            const float sn = u - __builtin_amdgcn_fmed3f(u, -tc, tc);
                            Y[rt][ct][r] = fmaf(bk1, sn, Y[rt][ct][r]);
                            X[rt][ct][r] = nbn * sn;
                        }
                    } else {
                        floatx16 spv;
                        if (ut < SPR) {
                            spv = sp[ut < SPR ? ut : 0];
                        } else {
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const float4 t4 = Sl[((w * SPL + ut - SPR) * 4 + q) * 64 + ln];
                                spv[4 * q] = t4.x;
                                spv[4 * q + 1] = t4.y;
                                spv[4 * q + 2] = t4.z;
                                spv[4 * q + 3] = t4.w;
                            }
                        }
                        // s_k = u - med3(u, -tau, tau); v = s_k + beta_k (s_k - s_{k-1}).
                        // With y^ in registers v is taken as (1 + beta_k) s_k -
                        // beta_k s_{k-1} (four VALU operations); the n = 1024
                        // classes keep the form whose temporaries do not spill
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const float u = X[rt][ct][r];
                            if constexpr (YREG) {
                                const float m = nbk * spv[r];
                                spv[r] = u - __builtin_amdgcn_fmed3f(u, -tc, tc);
                                X[rt][ct][r] = fmaf(bk1, spv[r], m);
                            } else {
                                const float sn = u - __builtin_amdgcn_fmed3f(u, -tc, tc);
                                X[rt][ct][r] = fmaf(bk, sn - spv[r], sn);
                                spv[r] = sn;
                            }
                        }
                        if (ut < SPR) {
                            sp[ut < SPR ? ut : 0] = spv;
                        } else {
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                Sl[((w * SPL + ut - SPR) * 4 + q) * 64 + ln] =
                                    make_float4(spv[4 * q], spv[4 * q + 1], spv[4 * q + 2], spv[4 * q + 3]);
                        }
                    }
                    const floatx16& vn = PP ? Y[rt][ct] : X[rt][ct];
                    Vb[((2 * gg) * CT + ct) * 64 + ln] = pack_bf16(vn, 0);
                    Vb[((2 * gg + 1) * CT + ct) * 64 + ln] = pack_bf16(vn, 1);
                }
            }
            __syncthreads();
          }
        }
        // ---- write s_T (PP: in vv after an odd number of iterations, else in pp)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int b = ct * 32 + col;
                const int ut = rt * CT + ct;
                floatx16 a;
                if constexpr (PP) {
                    a = (T & 1) ? vv[rt][ct] : pp[rt][ct];
                } else if (ut < SPR) {
                    a = sp[ut < SPR ? ut : 0];
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float4 t4 = Sl[((w * SPL + ut - SPR) * 4 + q) * 64 + ln];
                        a[4 * q] = t4.x;
                        a[4 * q + 1] = t4.y;
                        a[4 * q + 2] = t4.z;
                        a[4 * q + 3] = t4.w;
                    }
                }
                if (b < tl.nblk) {
                    float* dst = tl.s + (size_t)b * N + (w * RT + rt) * 32 + 4 * h;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        *reinterpret_cast<float4*>(dst + 8 * q) =
                            make_float4(a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]);
                }
            }
    }
}

template <int N, int MP, int CT, int W, int PF, int PA, int SPL, int OCC, int NL, int OPT = 0>
static void launch_class(const FusedTile* tiles, const int* qoff, const int* queue, int* counters,
                         int grid, hipStream_t st) {
    static_assert(W * OCC % 4 == 0 && W * OCC <= 32, "waves per CU");
    constexpr size_t kFT = ((MP / 32) * CT + W - 1) / W;
    constexpr size_t kNL = NL < 0 ? -NL : NL;
    constexpr size_t kOp = (OPT & 2) ? ((size_t)(MP / 32) * (N / 16) + (size_t)(N / 32) * (MP / 16)) * 1024
                           : (OPT & 8) ? (size_t)(N / 32) * (MP / 16) * 1024
                                       : 0;   // LDS-resident operator (or its adjoint layout)
    constexpr size_t kLds = (size_t)(N / 16) * CT * 1024 + (size_t)(MP / 16) * CT * 1024 +
                            (size_t)W * SPL * 4096 + (size_t)W * kFT * kNL * 1024 + kOp;
    static_assert((kLds + 64) * OCC <= 160 * 1024, "LDS of OCC workgroups exceeds a CU");
    const size_t lds = kLds;
    auto* fn = &fista_bf16_kernel<N, MP, CT, W, PF, PA, SPL, OCC, NL, OPT>;
    ensure_lds_limit<&fista_bf16_kernel<N, MP, CT, W, PF, PA, SPL, OCC, NL, OPT>>(lds);
    fn<<<dim3(grid), dim3(64 * W), lds, st>>>(tiles, qoff, queue, counters);
    CSV_HIP(hipGetLastError());
}

// Kernel variants per (n, Mp) class: column tiles CT, waves W, ring depths
// (forward, adjoint), LDS-resident state tiles and workgroups per CU.
// Variant 0 is the default; the autotuner (csv_autotune) times them and
// records a choice.
#define CSV_VG(NN, MM, CT, W, PF, PA, SPL, OCC, NLS, SUFFIX)                               \
    FusedVariant {                                                                         \
        "ct" #CT "_w" #W "_pf" #PF "_pa" #PA "_spl" #SPL "_o" #OCC SUFFIX, CT, OCC,         \
            &launch_class<NN, MM, CT, W, PF, PA, SPL, OCC, NLS>                             \
    }
#define CSV_V(NN, MM, CT, W, PF, PA, SPL, OCC) CSV_VG(NN, MM, CT, W, PF, PA, SPL, OCC, 0, "")
#define CSV_VY(NN, MM, CT, W, PF, PA, SPL, OCC)                                             \
    FusedVariant {                                                                         \
        "ct" #CT "_w" #W "_pf" #PF "_pa" #PA "_spl" #SPL "_o" #OCC "_yreg", CT, OCC,        \
            &launch_class<NN, MM, CT, W, PF, PA, SPL, OCC, 0, 1>                            \
    }
#define CSV_VOL(NN, MM, CT, W, PF, PA, OCC)                                                 \
    FusedVariant {                                                                         \
        "ct" #CT "_w" #W "_pf" #PF "_pa" #PA "_spl0_o" #OCC "_yreg_oplds", CT, OCC,         \
            &launch_class<NN, MM, CT, W, PF, PA, 0, OCC, 0, 3>                              \
    }
#define CSV_VL(NN, MM, CT, W, PF, PA, SPL, OCC, NL) \
    CSV_VG(NN, MM, CT, W, PF, PA, SPL, OCC, NL, "_lds" #NL)
#define CSV_VLI(NN, MM, CT, W, PF, PA, SPL, OCC, NL) \
    CSV_VG(NN, MM, CT, W, PF, PA, SPL, OCC, -NL, "_ldsi" #NL)
#define CSV_VOA(NN, MM, CT, W, PF, PA, OCC, OPTV, SUFFIX)                                  \
    FusedVariant {                                                                         \
        "ct" #CT "_w" #W "_pf" #PF "_pa" #PA "_spl0_o" #OCC SUFFIX, CT, OCC,                \
            &launch_class<NN, MM, CT, W, PF, PA, 0, OCC, 0, OPTV>                           \
    }
#define CSV_VLIP(NN, MM, CT, W, PF, PA, OCC, NL)                                            \
    FusedVariant {                                                                         \
        "ct" #CT "_w" #W "_pf" #PF "_pa" #PA "_spl0_o" #OCC "_ldsi" #NL "_pp", CT, OCC,     \
            &launch_class<NN, MM, CT, W, PF, PA, 0, OCC, -NL, 4>                            \
    }

struct ClassEntry {
    int n, Mp;
    std::vector<FusedVariant> v;
    int choice;
};

static std::vector<ClassEntry>& class_table() {
    static std::vector<ClassEntry> t = {
        {256, 32,
         {CSV_VOL(256, 32, 2, 4, 4, 2, 2), CSV_VOL(256, 32, 2, 4, 8, 2, 2),
          CSV_VOL(256, 32, 1, 4, 4, 2, 3), CSV_VOL(256, 32, 4, 8, 4, 2, 1),
          CSV_VOL(256, 32, 4, 8, 8, 2, 1), CSV_VY(256, 32, 2, 4, 4, 2, 0, 2),
          CSV_VY(256, 32, 1, 4, 4, 2, 0, 3), CSV_V(256, 32, 1, 4, 4, 2, 0, 3)},
         0},
        {256, 64,
         {CSV_VOL(256, 64, 4, 8, 4, 2, 1), CSV_VOL(256, 64, 4, 8, 8, 2, 1),
          CSV_VOL(256, 64, 4, 8, 8, 4, 1), CSV_VOL(256, 64, 2, 8, 8, 2, 1),
          CSV_VOL(256, 64, 2, 8, 16, 2, 1), CSV_VY(256, 64, 2, 4, 4, 2, 0, 2),
          CSV_V(256, 64, 2, 4, 4, 2, 0, 2)},
         0},
        {256, 96,
         {CSV_VOL(256, 96, 2, 8, 4, 3, 1), CSV_VOL(256, 96, 2, 8, 8, 3, 1),
          CSV_VOL(256, 96, 2, 8, 8, 2, 1), CSV_VOL(256, 96, 2, 8, 4, 2, 1),
          CSV_VOL(256, 96, 2, 8, 16, 3, 1), CSV_VY(256, 96, 2, 4, 2, 2, 0, 2),
          CSV_VY(256, 96, 1, 4, 2, 2, 0, 3), CSV_V(256, 96, 1, 4, 2, 2, 0, 3)},
         0},
        {256, 128,
         {CSV_VOA(256, 128, 2, 8, 8, 4, 1, 13, "_yreg_opadj_pp"),
          CSV_VY(256, 128, 2, 4, 2, 2, 0, 2),
          CSV_VOA(256, 128, 2, 8, 8, 8, 1, 13, "_yreg_opadj_pp"),
          CSV_VOA(256, 128, 2, 8, 8, 2, 1, 13, "_yreg_opadj_pp"),
          CSV_VOA(256, 128, 2, 8, 16, 4, 1, 13, "_yreg_opadj_pp"),
          CSV_VOA(256, 128, 2, 8, 8, 4, 1, 9, "_yreg_opadj"),
          CSV_VOA(256, 128, 2, 8, 4, 2, 1, 9, "_yreg_opadj"),
          CSV_V(256, 128, 1, 4, 2, 2, 0, 3),
          CSV_V(256, 128, 2, 4, 2, 2, 0, 2), CSV_VOL(256, 128, 1, 4, 2, 2, 1),
          CSV_VY(256, 128, 1, 4, 2, 2, 0, 3), CSV_V(256, 128, 2, 8, 4, 2, 0, 1),
          CSV_V(256, 128, 4, 8, 4, 2, 0, 1)},
         0},
        {1024, 32,
         {CSV_VLIP(1024, 32, 1, 8, 4, 2, 1, 8), CSV_VLI(1024, 32, 1, 8, 4, 2, 0, 1, 8),
          CSV_V(1024, 32, 1, 8, 4, 2, 0, 1), CSV_V(1024, 32, 1, 8, 4, 2, 2, 1),
          CSV_VL(1024, 32, 1, 8, 4, 2, 0, 1, 8)},
         0},
        {1024, 64,
         {CSV_VLIP(1024, 64, 1, 8, 4, 2, 1, 8), CSV_VLI(1024, 64, 1, 8, 4, 2, 0, 1, 8),
          CSV_V(1024, 64, 1, 8, 4, 2, 0, 1), CSV_V(1024, 64, 1, 8, 4, 2, 2, 1),
          CSV_VL(1024, 64, 1, 8, 4, 2, 0, 1, 8)},
         0},
        {1024, 128,
         {CSV_VLIP(1024, 128, 1, 8, 4, 2, 1, 8), CSV_VLI(1024, 128, 1, 8, 4, 2, 0, 1, 8),
          CSV_V(1024, 128, 1, 8, 4, 2, 0, 1), CSV_V(1024, 128, 1, 8, 4, 2, 2, 1),
          CSV_VL(1024, 128, 1, 8, 4, 2, 0, 1, 8)},
         0},
        {1024, 224,
         {CSV_VLIP(1024, 224, 1, 8, 4, 2, 1, 8), CSV_VLI(1024, 224, 1, 8, 4, 2, 0, 1, 8),
          CSV_V(1024, 224, 1, 8, 4, 2, 0, 1), CSV_V(1024, 224, 1, 8, 4, 2, 2, 1),
          CSV_VL(1024, 224, 1, 8, 4, 2, 0, 1, 8)},
         0},
        {1024, 256,
         {CSV_VLIP(1024, 256, 1, 8, 4, 2, 1, 8), CSV_VLI(1024, 256, 1, 8, 4, 2, 0, 1, 8),
          CSV_V(1024, 256, 1, 8, 4, 2, 0, 1), CSV_V(1024, 256, 1, 8, 4, 2, 2, 1),
          CSV_V(1024, 256, 1, 8, 8, 2, 2, 1), CSV_V(1024, 256, 1, 8, 4, 2, 1, 1),
          CSV_VL(1024, 256, 1, 8, 4, 2, 0, 1, 8),
          FusedVariant{"q8_w8_pf2x2_pa2x2", 1, 1, &launch_fista_q8_m256}},
         0},
        {1024, 416,
         {CSV_V(1024, 416, 1, 8, 2, 2, 2, 1), CSV_V(1024, 416, 1, 8, 2, 2, 0, 1),
          CSV_V(1024, 416, 1, 8, 4, 2, 2, 1)},
         0},
    };
    return t;
}
#undef CSV_V
#undef CSV_VY
#undef CSV_VOL
#undef CSV_VL
#undef CSV_VLI
#undef CSV_VLIP
#undef CSV_VOA
#undef CSV_VG

static ClassEntry* find_class(int n, int Mp) {
    for (auto& c : class_table())
        if (c.n == n && c.Mp == Mp) return &c;
    return nullptr;
}

bool fused_class_supported(int n, int Mp) { return find_class(n, Mp) != nullptr; }

const std::vector<FusedVariant>& fused_variants(int n, int Mp) {
    ClassEntry* c = find_class(n, Mp);
    CSV_REQUIRE(c, CSV_EUNSUPPORTED,
                "fused BF16 recovery has no kernel for n=" + std::to_string(n) +
                    ", padded M=" + std::to_string(Mp));
    return c->v;
}

// The choice of a class is process-wide and may be set (csv_autotune,
// csv_autotune_load) while other threads decode: read and written atomically.
int fused_choice(int n, int Mp) {
    ClassEntry* c = find_class(n, Mp);
    return c ? __atomic_load_n(&c->choice, __ATOMIC_RELAXED) : 0;
}

void set_fused_choice(int n, int Mp, int idx) {
    ClassEntry* c = find_class(n, Mp);
    CSV_REQUIRE(c && idx >= 0 && idx < (int)c->v.size(), CSV_EINVAL, "no such kernel variant");
    __atomic_store_n(&c->choice, idx, __ATOMIC_RELAXED);
}

std::vector<std::pair<int, int>> fused_classes() {
    std::vector<std::pair<int, int>> out;
    for (auto& c : class_table()) out.push_back({c.n, c.Mp});
    return out;
}

int fused_tile_blocks(int n, int Mp) {
    const auto& v = fused_variants(n, Mp);
    return 32 * v[fused_choice(n, Mp)].ct;
}

// Compute units of the current device (cached per device).
int device_cus() {
    static std::atomic<int> cus[64];
    int dev = 0;
    CSV_HIP(hipGetDevice(&dev));
    CSV_REQUIRE(dev >= 0 && dev < 64, CSV_EINVAL, "device index out of range");
    int c = cus[dev].load(std::memory_order_relaxed);
    if (c <= 0) {
        CSV_HIP(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
        CSV_REQUIRE(c > 0, CSV_EHIP, "device reports no compute units");
        cus[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

void launch_fista_bf16_class(int n, int Mp, const FusedTile* tiles, const int* qoff,
                             const int* queue, int* counters, int count, hipStream_t st,
                             int variant) {
    const auto& v = fused_variants(n, Mp);
    const int idx = variant >= 0 ? variant : fused_choice(n, Mp);
    CSV_REQUIRE(idx < (int)v.size(), CSV_EINVAL, "no such kernel variant");
    const int grid = std::min(count, device_cus() * v[idx].occ);
    v[idx].launch(tiles, qoff, queue, counters, grid, st);
}

}  // namespace csv
