// Fused BF16 total-variation recovery for 16 x 16 blocks (the TVAL3-style
// solver of Section 4, reference [14]): all T iterations of a tile of 32
// blocks run inside one workgroup, both Phi products on MFMA, the iterates
// and multipliers in FP32 registers.  The iteration is that of k_tv.hip
// (nu <- nu + beta (D x - w_prev); w = shrink(D x + nu / beta, lam / beta);
// P = nu + beta (D x - w); x <- x - alpha (Phi^T (Phi x - y^) + D^T P),
// alpha = 1 / (L + 8 beta)), carried in mu = nu - beta w so that only x and
// mu persist:
//   nu = mu + beta D x;  w = shrink(D x + nu / beta, lam / beta);
//   mu <- nu - beta w;   P = mu + beta D x;  x <- x - alpha (G + D^T P),
// with D the forward differences inside the block (Neumann boundary); D x of
// the dual step is kept for the primal step.  The residual goes to LDS as
// alpha (y^ - Phi x) and the adjoint accumulator starts at x, so the Phi^T
// product ends at x - alpha G.
//
// Layout.  Eight waves; wave w owns pixel group w (pixels 32 w .. 32 w + 31 =
// image rows 2 w and 2 w + 1 of every block) in the 32x32 MFMA accumulator
// layout: lane l holds block l % 32; register r holds pixel
// rho = 8 (r / 4) + 4 h + r % 4 of the group (h = l / 32), i.e. image row
// 2 w + (r >> 3) and column 8 ((r >> 2) & 1) + 4 h + (r & 3).  The stencils
// therefore need:
//   right neighbour (column + 1): register r + 1 when r & 3 < 3; otherwise
//     the partner lane l ^ 32 (register r - 3 from lane half 0, register
//     r + 1 from lane half 1 when column 7), none at column 15;
//   left neighbour (column - 1): register r - 1 when r & 3 > 0; otherwise the
//     partner lane (register r + 3 from lane half 1, register r - 1 from
//     lane half 0 when column 8), none at column 0;
//   lower neighbour (row + 1): register r + 8 for the group's first row; the
//     next wave's first row (through LDS) for its second; none at row 15;
//   upper neighbour (row - 1): register r - 8 for the second row; the
//     previous wave's second row (through LDS) for the first; none at row 0.
// Per iteration: the dual step (registers; P of the group's last row to LDS),
// the forward product Phi V (V = bf16 x from LDS) with R = Phi V - y^ to LDS,
// barrier, the adjoint G = Phi^T R for the wave's group, the primal step, V
// and the group's first row of x to LDS, barrier.  LDS rows read before a
// barrier are rewritten only after the next one.
#include <algorithm>
#include <type_traits>

#include "fused_common.h"
#include "tv_step.h"

namespace csv {

// Values of the partner lane (l ^ 32) at registers 0, 4, 8, 12 (c = 0) or
// 3, 7, 11, 15 (c = 3).
__device__ inline floatx4 partner4(const floatx16& t, int first) {
    floatx4 o;
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = __shfl_xor(t[first + 4 * i], 32);
    return o;
}

// Right neighbour of every register (0 where none); hi: lane half 1.
// Branch-free: the lane half only selects between two values.
__device__ inline floatx16 right_of(const floatx16& t, bool hi) {
    const floatx4 p0 = partner4(t, 0);   // partner registers 0, 4, 8, 12
    floatx16 o;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int c = r & 3, q = (r >> 2) & 1;
        if (c < 3) {
            o[r] = t[r + 1];
        } else {
            // half 0: partner register r - 3; half 1: partner register r + 1
            // (column 7), none at column 15
            const float from_hi = q == 0 ? p0[(r + 1) >> 2] : 0.f;
            o[r] = hi ? from_hi : p0[(r - 3) >> 2];
        }
    }
    return o;
}

// Left neighbour of every register (0 where none).
__device__ inline floatx16 left_of(const floatx16& t, bool hi) {
    const floatx4 p3 = partner4(t, 3);   // partner registers 3, 7, 11, 15
    floatx16 o;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int c = r & 3, q = (r >> 2) & 1;
        if (c > 0) {
            o[r] = t[r - 1];
        } else {
            // half 1: partner register r + 3; half 0: partner register r - 1
            // (column 8), none at column 0
            const float from_lo = q == 1 ? p3[(r - 1) >> 2] : 0.f;
            o[r] = hi ? p3[(r + 3) >> 2] : from_lo;
        }
    }
    return o;
}

// Register r is in the last column (15) / the first column (0) of the block.
__device__ inline bool last_col(int r, bool hi) { return (r & 7) == 7 && hi; }
__device__ inline bool first_col(int r, bool hi) { return (r & 7) == 0 && !hi; }

// D x of the wave's group: horizontal and vertical forward differences.
__device__ inline void grad_group(const floatx16& x, const float* xrow, int w, int ln, bool hi,
                                  floatx16& dh, floatx16& dv) {
    const floatx16 xr = right_of(x, hi);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        dh[r] = last_col(r, hi) ? 0.f : xr[r] - x[r];
        float down;
        if (r < 8)
            down = x[r + 8];
        else
            down = w + 1 < 8 ? xrow[((w + 1) * 8 + (r - 8)) * 64 + ln] : x[r];   // row 15: none
        dv[r] = down - x[r];
    }
}

// The forward waves keep their y^ rows of the tile in registers, scaled by
// alpha, for all T iterations (the residual epilogue is one FMA per value).
// OPL: both layouts of Phi (M_p x 256 bf16 fragments) are copied into LDS
// when a tile's operator differs from the previous tile's, and every
// iteration reads them there instead of from L2.
template <int MP, int kPF, int kPA, int OCC, bool OPL>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2 * OCC)))
void tv_bf16_kernel(const FusedTile* __restrict__ tiles, const int* __restrict__ qoff,
                    const int* __restrict__ queue, int* __restrict__ counters) {
    constexpr int N = 256, W = 8, CT = 1;
    constexpr int OFW = (MP / 32) * (N / 16) * 64, OFA = (N / 32) * (MP / 16) * 64;   // u16x8
    using PT = std::conditional_t<OPL, u16x8, gu16x8>;
    constexpr int KSF = N / 16, KSA = MP / 16;
    constexpr int TT = MP / 32;                  // forward output tiles (one per wave w < TT)
    static_assert(TT <= W, "one forward tile per wave");
    static_assert(KSF % kPF == 0 && KSA % kPA == 0 && KSA >= kPA, "ring depths");
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    u16x8* Vb = reinterpret_cast<u16x8*>(lds);                              // [KSF][64]
    u16x8* Rb = reinterpret_cast<u16x8*>(lds + (size_t)KSF * 1024);         // [KSA][64]
    float* xrow = reinterpret_cast<float*>(lds + (size_t)(KSF + KSA) * 1024);   // [W][8][64]
    float* prow = xrow + W * 8 * 64;                                        // [W][8][64]
    u16x8* Ol = reinterpret_cast<u16x8*>(prow + W * 8 * 64);                // OPL: [OFW][OFA]
    __shared__ int s_tile;
    const void* ol_src = nullptr;

    const int tid = threadIdx.x, ln = tid & 63, h = ln >> 5, col = ln & 31;
    // the wave index is uniform across the wave: keep it in a scalar register
    // so that conditions on it are scalar branches
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool fwd = w < TT, hi = h != 0;

    for (;;) {
        if (tid == 0) s_tile = next_tile(qoff, queue, counters);
        __syncthreads();
        const int t_id = s_tile;
        __syncthreads();
        if (t_id < 0) break;
        const FusedTile tl = tiles[t_id];
        const PT* ffwd;
        const PT* fadj;
        if constexpr (OPL) {
            // every wave is past the previous tile (barriers above)
            if (tl.frag_fwd != ol_src) {
                const gu16x8* gf = as_global<const gu16x8>(tl.frag_fwd);
                const gu16x8* gad = as_global<const gu16x8>(tl.frag_adj);
                for (int i = tid; i < OFW; i += 512) Ol[i] = gf[i];
                for (int i = tid; i < OFA; i += 512) Ol[OFW + i] = gad[i];
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
        const float lam = col < tl.nblk ? tl.lam[col] : 0.f;
        const float beta = tv_beta(lam);
        const float inv_beta = 1.f / beta, thr = lam / beta;
        const float alpha = tv_alpha(tl.lip[0], beta);
        const int T = tl.T;
        floatx16 yv = {};   // alpha y^ of this wave's forward tile (rows 32 w ..)
        if (fwd && col < tl.nblk) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                yv[r] = yg[(size_t)col * MP + w * 32 + 8 * (r / 4) + 4 * h + (r % 4)] * alpha;
        }

        floatx16 x = {}, mh = {}, mv = {};
        {
            const u16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
            Vb[(2 * w) * 64 + ln] = z;
            Vb[(2 * w + 1) * 64 + ln] = z;
#pragma unroll
            for (int r = 0; r < 8; ++r) xrow[(w * 8 + r) * 64 + ln] = 0.f;
        }
        u16x8 af[kPF][1];
        u16x8 aa[kPA][1];
        if (fwd) load_fwd_head<N, MP, CT, 1, W, kPF>(af, ffwd, w, ln);
        __syncthreads();

        for (int k = 0; k < T; ++k) {
            // ---- dual step: nu = mu + beta D x, w = shrink, mu = nu - beta w
            // (D x stays in registers for the primal step)
            floatx16 dh, dv;
            {
                grad_group(x, xrow, w, ln, hi, dh, dv);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float n1 = fmaf(beta, dh[r], mh[r]);
                    const float n2 = fmaf(beta, dv[r], mv[r]);
                    const float vh = fmaf(n1, inv_beta, dh[r]), vv = fmaf(n2, inv_beta, dv[r]);
                    // shrink factor max(|v| - thr, 0) / |v| = max(1 - thr rsq(|v|^2), 0):
                    // |v| = 0 gives rsq = inf and the max keeps 0 (also for thr = 0,
                    // where the product is NaN and max returns the other operand)
                    const float m2 = fmaf(vh, vh, vv * vv);
                    const float sc = fmaxf(fmaf(-thr, __builtin_amdgcn_rsqf(m2), 1.f), 0.f);
                    mh[r] = fmaf(-beta, sc * vh, n1);
                    mv[r] = fmaf(-beta, sc * vv, n2);
                }
#pragma unroll
                for (int r = 8; r < 16; ++r)   // P_v of the group's last row, for the next wave
                    prow[(w * 8 + (r - 8)) * 64 + ln] = fmaf(beta, dv[r], mv[r]);
            }
            // ---- forward Phi V, R = Phi V - y^ (waves w < TT)
            if (fwd) {
                floatx16 acc[1];
                forward_tiles<N, MP, CT, 1, 1, W, kPF, kPA>(af, aa, acc, ffwd, fadj, Vb, w, ln, 0, w);
                // R' = alpha (y^ - Phi V): the adjoint started at x ends at x - alpha G
                store_residual<MP, CT, true, true>(acc[0], yv, yg, tl.nblk, w, 0, ln, Rb, alpha);
            } else {
#pragma unroll
                for (int p = 0; p < kPA; ++p) aa[p][0] = fadj[((size_t)w * KSA + p) * 64 + ln];
            }
            __syncthreads();
            // ---- adjoint for group w: g = x - alpha Phi^T (Phi x - y^)
            floatx16 g = x;
#pragma unroll 1
            for (int ks0 = 0; ks0 < KSA - kPA; ks0 += kPA) {
#pragma unroll
                for (int j = 0; j < kPA; ++j) {
                    const int ks = ks0 + j;
                    const bf16x8 b = __builtin_bit_cast(bf16x8, Rb[ks * 64 + ln]);
                    g = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, aa[j][0]), b,
                                                               g, 0, 0, 0);
                    aa[j][0] = fadj[((size_t)w * KSA + ks + kPA) * 64 + ln];
                }
            }
#pragma unroll
            for (int j = 0; j < kPA; ++j) {
                const int ks = KSA - kPA + j;
                const bf16x8 b = __builtin_bit_cast(bf16x8, Rb[ks * 64 + ln]);
                g = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, aa[j][0]), b, g,
                                                           0, 0, 0);
            }
            if (fwd) load_fwd_head<N, MP, CT, 1, W, kPF>(af, ffwd, w, ln);
            // ---- primal step: P = mu + beta D x, x <- x - alpha (G + D^T P)
            {
                floatx16 ph, pv;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    ph[r] = fmaf(beta, dh[r], mh[r]);
                    pv[r] = fmaf(beta, dv[r], mv[r]);
                }
                const floatx16 pl = left_of(ph, hi);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    float dt = last_col(r, hi) ? 0.f : -ph[r];
                    dt += first_col(r, hi) ? 0.f : pl[r];
                    if (r < 8 || w + 1 < W) dt -= pv[r];   // rows below 15
                    if (r >= 8)
                        dt += pv[r - 8];
                    else if (w > 0)
                        dt += prow[((w - 1) * 8 + r) * 64 + ln];
                    x[r] = fmaf(-alpha, dt, g[r]);
                }
            }
            Vb[(2 * w) * 64 + ln] = pack_bf16(x, 0);
            Vb[(2 * w + 1) * 64 + ln] = pack_bf16(x, 1);
#pragma unroll
            for (int r = 0; r < 8; ++r) xrow[(w * 8 + r) * 64 + ln] = x[r];
            __syncthreads();
        }
        // ---- write x (pixel-domain residual, row-major in the block)
        const int b = col;
        if (b < tl.nblk) {
            float* dst = tl.s + (size_t)b * N + w * 32 + 4 * h;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<float4*>(dst + 8 * q) =
                    make_float4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
        }
    }
}

template <int MP, int PF, int PA, int OCC>
static void launch_tv_class(const FusedTile* tiles, const int* qoff, const int* queue,
                            int* counters, int grid, hipStream_t st) {
    // the operator joins V, R and the stencil rows in LDS when it fits (M_p <= 96)
    constexpr size_t base = (size_t)16 * 1024 + (size_t)(MP / 16) * 1024 + 2 * 8 * 8 * 64 * 4;
    constexpr size_t op = ((size_t)(MP / 32) * 16 + (size_t)8 * (MP / 16)) * 1024;
    constexpr bool OPL = (base + op + 64) * OCC <= 160 * 1024;
    constexpr size_t lds = base + (OPL ? op : 0);
    static_assert((lds + 64) * OCC <= 160 * 1024, "LDS of OCC workgroups exceeds a CU");
    auto* fn = &tv_bf16_kernel<MP, PF, PA, OCC, OPL>;
    ensure_lds_limit<&tv_bf16_kernel<MP, PF, PA, OCC, OPL>>(lds);
    fn<<<dim3(grid), dim3(512), lds, st>>>(tiles, qoff, queue, counters);
    CSV_HIP(hipGetLastError());
}

bool tv_class_supported(int n, int Mp) {
    return n == 256 && (Mp == 32 || Mp == 64 || Mp == 96 || Mp == 128);
}

void launch_tv_bf16_class(int n, int Mp, const FusedTile* tiles, const int* qoff,
                          const int* queue, int* counters, int count, int cus, hipStream_t st) {
    CSV_REQUIRE(tv_class_supported(n, Mp), CSV_EUNSUPPORTED,
                "fused BF16 TV recovery has no kernel for n=" + std::to_string(n) +
                    ", padded M=" + std::to_string(Mp));
    constexpr int OCC = 1;
    const int grid = std::min(count, cus * OCC);
    switch (Mp) {
        case 32: launch_tv_class<32, 4, 2, OCC>(tiles, qoff, queue, counters, grid, st); break;
        case 64: launch_tv_class<64, 4, 2, OCC>(tiles, qoff, queue, counters, grid, st); break;
        case 96: launch_tv_class<96, 4, 2, OCC>(tiles, qoff, queue, counters, grid, st); break;
        default: launch_tv_class<128, 4, 2, OCC>(tiles, qoff, queue, counters, grid, st); break;
    }
}

}  // namespace csv
