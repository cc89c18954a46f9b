// Fused BF16 recovery at n = 1024 (32 x 32 blocks) that streams the integer
// measurement matrix Q instead of the dense operator A = s_phi Q Psi.  The
// 2-D DCT Psi (X = C^T S C) is applied inside the workgroup on the matrix
// cores, so every iteration of a tile of 32 blocks reads Q twice as int8
// (forward and adjoint fragment orders, M_p n bytes each) instead of A twice
// as bf16: half the operator bytes, for 25% more MFMA work.
//
// Ownership.  Wave w = (s_w, q_w, h_w) (bits 2, 1, 0) owns the four indices
// O_w = {16 s_w + 8 q_w + 4 h_w + t, t < 4} of a 32-index DCT axis; these
// are elements 4 q_w .. 4 q_w + 3 of lane half h_w in K step s_w of a
// 32x32x16 MFMA fragment (kappa order, fused_common.h), so a wave's share of
// a fragment is one 8-byte LDS store.  The iterates of coefficient (k, l),
// c = 32 k + l, live with the wave owning l, as FP32 accumulator tiles
// V^l[k][b] (rows k, columns = the tile's blocks b).
//
// One iteration (C[a][b] the DCT table, R'' = s_phi (y - A v) / L):
//   F1   Y^l[i] = sum_k C[k][i] V^l[k]        own l, from registers
//        Y -> LDS in [i][l] fragment order                     barrier A
//   F2   X_i[j] = sum_l C[l][j] Y^l[i]        own i; X -> LDS as the
//        forward product's B fragments (pixel p = 32 i + j)    barrier B
//   fwd  P = s_phi Q X for M tile w; R'' -> LDS                barrier C
//   adj  Z_i[j] = sum_m Q[m][32 i + j] R''[m]  own i
//   A1   W_i[l] = sum_j C[l][j] Z_i[j]; W -> LDS in [l][i] order barrier D
//   A2   u^l[k] = V^l[k] + sum_i C[k][i] W_i[l]  own l (accumulators start
//        at v), then the threshold and momentum step on u^l.
// Q is stored as the byte q + 64 (q in [-32, 32]); v_perm pairs it with
// 0x43 into the bf16 of 128 + (q + 64), so the products see q + 192, and
// 192 times the column sums of the bf16 X and R'' are subtracted.
#include <algorithm>

#include "fused_common.h"

namespace csv {

namespace {

constexpr int kQN = 1024, kQKSF = 64;   // n and forward K steps

__device__ inline int rho_row(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 gu32x4;

// Eight biased bytes (q + 64) -> eight bf16 of q + 192, in byte order.
__device__ inline bf16x8 widen_q(u32x2 w) {
    const unsigned k43 = 0x43434343u;
    uint4 o;
    o.x = __builtin_amdgcn_perm(k43, w.x, 0x04010400u);
    o.y = __builtin_amdgcn_perm(k43, w.x, 0x04030402u);
    o.z = __builtin_amdgcn_perm(k43, w.y, 0x04010400u);
    o.w = __builtin_amdgcn_perm(k43, w.y, 0x04030402u);
    return __builtin_bit_cast(bf16x8, o);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// two floats -> one dword of two bf16 (one v_cvt_pk_bf16_f32)
__device__ inline unsigned cvt2(float a, float b) {
    const f32x2 v = {a, b};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}

// acc + the sum of the 8 bf16 of a fragment (four dot products with ones)
__device__ inline float frag_sum(const u16x8& f, float acc) {
    const uint4 d = __builtin_bit_cast(uint4, f);
    const bf16x2 one = {(__bf16)1.0f, (__bf16)1.0f};
    acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, d.x), one, acc, false);
    acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, d.y), one, acc, false);
    acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, d.z), one, acc, false);
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, d.w), one, acc, false);
}

__device__ inline floatx16 mma(const bf16x8& a, const u16x8& b, const floatx16& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

}  // namespace

// Two K steps (s = 0, 1 of one 32-group g) per lane and 16-byte load:
// qb_fwd[mt][g][lane][8 s + e] = Q[32 mt + lane % 32][32 g + kappa(s, lane / 32, e)] + 64
// qb_adj[pg][g][lane][8 s + e] = Q[32 g + kappa(s, lane / 32, e)][32 pg + lane % 32] + 64
__global__ void q8_frag_layout_kernel(const int8_t* __restrict__ q, int n, int Mp,
                                      uint8_t* __restrict__ fwd, uint8_t* __restrict__ adj) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)Mp * n) return;
    const int e = (int)(idx & 7), s = (int)((idx >> 3) & 1), lane = (int)((idx >> 4) & 63);
    const size_t pair = idx >> 10;
    const int h = lane >> 5, i = lane & 31;
    {
        const int g = (int)(pair % (n / 32)), mt = (int)(pair / (n / 32));
        const int row = mt * 32 + i, col = 32 * g + kappa(s, h, e);
        fwd[idx] = (uint8_t)(q[(size_t)row * n + col] + 64);
    }
    {
        const int g = (int)(pair % (Mp / 32)), pg = (int)(pair / (Mp / 32));
        const int row = 32 * g + kappa(s, h, e), col = pg * 32 + i;
        adj[idx] = (uint8_t)(q[(size_t)row * n + col] + 64);
    }
}

void launch_q8_frag_layout(Operator* op, hipStream_t st) {
    const size_t total = (size_t)op->Mp * op->n;
    q8_frag_layout_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st>>>(
        op->q, op->n, op->Mp, op->qb_fwd, op->qb_adj);
    CSV_HIP(hipGetLastError());
}

template <int MP, int kPF, int kPA>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
void fista_q8_kernel(const FusedTile* __restrict__ tiles, const int* __restrict__ qoff,
                     const int* __restrict__ queue, int* __restrict__ counters) {
    constexpr int TT = MP / 32, KSA = MP / 16;   // forward tiles, adjoint K steps
    constexpr int KPF2 = kQKSF / 2, KPA2 = KSA / 2;   // K-step pairs (one 16-byte load each)
    static_assert(MP % 32 == 0 && TT >= 1 && TT <= 8, "one forward M tile per wave at most");
    static_assert(KPF2 % kPF == 0 && KPA2 % kPA == 0 && KPF2 > kPF, "ring depth must divide the pairs");
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    u16x8* XW = reinterpret_cast<u16x8*>(lds);                 // X fragments [64][64] / W [32][2][64]
    u16x8* YX = reinterpret_cast<u16x8*>(lds + 65536);         // Y [32][2][64]
    u16x8* Rb = reinterpret_cast<u16x8*>(lds + 131072);        // R'' fragments [KSA][64]
    float* csum = reinterpret_cast<float*>(lds + 131072 + KSA * 1024);   // [8][32]
    float* rsum = csum + 256;                                             // [8][32]
    u16x8* Cf = reinterpret_cast<u16x8*>(rsum + 256);   // DCT fragments ct[0], ct[1], cn[0], cn[1] [4][64]
    __shared__ int s_tile;

    const int tid = threadIdx.x, w = tid >> 6, ln = tid & 63, h = ln >> 5, col = ln & 31;
    const int sw = (w >> 2) & 1, qw = (w >> 1) & 1, hw = w & 1;
    const int o0 = 16 * sw + 8 * qw + 4 * hw;   // owned indices o0 .. o0 + 3
    const bool fwd = w < TT;
    // a wave's 8-byte share of fragment (row index x, K step sw, lane (hw, col)):
    // uint2 index 256 x + share, written as two 4-byte halves (t = 0, 1 and t = 2, 3)
    const int share = (sw * 64 + hw * 32 + col) * 2 + qw;
    unsigned* YX1 = reinterpret_cast<unsigned*>(YX);
    unsigned* XW1 = reinterpret_cast<unsigned*>(XW);

    for (;;) {
        if (tid == 0) s_tile = next_tile(qoff, queue, counters);
        __syncthreads();
        // uniform: the descriptor and the tables it points to are then
        // read with scalar loads
        const int t_id = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (t_id < 0) break;
        const FusedTile tl = tiles[t_id];
        const gu32x4* qf = as_global<const gu32x4>(tl.qb_fwd);   // [TT][32][64] pairs
        const gu32x4* qa = as_global<const gu32x4>(tl.qb_adj);   // [32][KSA / 2][64] pairs
        const gfloat* yg = as_global<const gfloat>(tl.y);
        const gfloat* dct = as_global<const gfloat>(tl.dct);
        const float inv_l = (float)(1.0 / as_global<cdouble>(tl.lip)[0]);
        const float sphi = tl.s_phi, rscale = tl.s_phi * inv_l;
        const int T = tl.T, nblk = tl.nblk;
        const cfloat* __restrict__ beta = as_global<cfloat>(tl.beta);
        const float tau = col < nblk ? as_global<const gfloat>(tl.lam)[col] * inv_l : 0.f;
        // DCT fragments in LDS: ct[s] = A[i][k] = C[k][i], cn[s] = A[l][j] = C[l][j]
        if (w < 4) {
            const int s = w & 1;
            u16x8 f;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int kk = kappa(s, h, e);
                f[e] = __builtin_bit_cast(uint16_t, (__bf16)(w < 2 ? dct[kk * 32 + col] : dct[col * 32 + kk]));
            }
            Cf[w * 64 + ln] = f;
        }
        __syncthreads();
        auto ct = [&](int s) { return __builtin_bit_cast(bf16x8, Cf[s * 64 + ln]); };
        auto cn = [&](int s) { return __builtin_bit_cast(bf16x8, Cf[(2 + s) * 64 + ln]); };
        floatx16 vv[4], sp[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            vv[t] = floatx16{};
            sp[t] = floatx16{};
        }
        u32x4 rf[kPF], ra[kPA];   // rings of K-step pairs
        for (int k = 0; k < T; ++k) {
            // ---- F1: Y^l = C^T-contraction of V^l over k; Y -> LDS
            {
                const bf16x8 c0 = ct(0), c1 = ct(1);
#pragma unroll
                for (int tp = 0; tp < 2; ++tp) {   // bf16 pairs (t = 2 tp, 2 tp + 1): one 4-byte store each
                    floatx16 ya = mma(c0, pack_bf16(vv[2 * tp], 0), floatx16{});
                    ya = mma(c1, pack_bf16(vv[2 * tp], 1), ya);
                    floatx16 yb = mma(c0, pack_bf16(vv[2 * tp + 1], 0), floatx16{});
                    yb = mma(c1, pack_bf16(vv[2 * tp + 1], 1), yb);
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        YX1[(rho_row(r, h) * 256 + share) * 2 + tp] = cvt2(ya[r], yb[r]);
                }
            }
            __syncthreads();   // A
            // forward ring head: in flight during F2
            if (fwd) {
#pragma unroll
                for (int p = 0; p < kPF; ++p) rf[p] = qf[((size_t)w * KPF2 + p) * 64 + ln];
            }
            // ---- F2: X_i for own i; column sums of the bf16 X; X -> LDS
            {
                float cs = 0.f;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int i = o0 + t;
                    floatx16 x = mma(ct(0), YX[(2 * i) * 64 + ln], floatx16{});
                    x = mma(ct(1), YX[(2 * i + 1) * 64 + ln], x);
                    const u16x8 p0 = pack_bf16(x, 0), p1 = pack_bf16(x, 1);
                    XW[(2 * i) * 64 + ln] = p0;
                    XW[(2 * i + 1) * 64 + ln] = p1;
                    cs = frag_sum(p1, frag_sum(p0, cs));
                }
                cs += __shfl_xor(cs, 32);
                if (h == 0) csum[w * 32 + col] = cs;
            }
            __syncthreads();   // B
            // ---- forward product for M tile w: P = s_phi Q X, R'' = s_phi (y - P) / L
            if (fwd) {
                float colsum = 0.f;
#pragma unroll
                for (int v = 0; v < 8; ++v) colsum += csum[v * 32 + col];
                floatx16 acc;   // started at -192 colsum: the bias of the widened Q cancels
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[r] = -192.f * colsum;
#pragma unroll 1
                for (int g0 = 0; g0 < KPF2 - kPF; g0 += kPF) {
#pragma unroll
                    for (int j = 0; j < kPF; ++j) {
                        const u32x4 qq = rf[j];
                        rf[j] = qf[((size_t)w * KPF2 + g0 + j + kPF) * 64 + ln];
                        acc = mma(widen_q(qq.xy), XW[(2 * (g0 + j)) * 64 + ln], acc);
                        acc = mma(widen_q(qq.zw), XW[(2 * (g0 + j) + 1) * 64 + ln], acc);
                    }
                }
#pragma unroll
                for (int j = 0; j < kPF; ++j) {   // last pairs: the adjoint ring head goes in flight
                    const int g = KPF2 - kPF + j;
                    acc = mma(widen_q(rf[j].xy), XW[(2 * g) * 64 + ln], acc);
                    acc = mma(widen_q(rf[j].zw), XW[(2 * g + 1) * 64 + ln], acc);
                    if (j < kPA) ra[j] = qa[((size_t)(o0 + j / KPA2) * KPA2 + j % KPA2) * 64 + ln];
                }
#pragma unroll
                for (int j = kPF; j < kPA; ++j)
                    ra[j] = qa[((size_t)(o0 + j / KPA2) * KPA2 + j % KPA2) * 64 + ln];
                floatx16 rr;
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) {
                    float yq[4] = {0.f, 0.f, 0.f, 0.f};
                    if (col < nblk) {
                        const gfloat* yp = yg + (size_t)col * MP + w * 32 + 8 * q4 + 4 * h;
                        yq[0] = yp[0];
                        yq[1] = yp[1];
                        yq[2] = yp[2];
                        yq[3] = yp[3];
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float pm = sphi * acc[4 * q4 + e];
                        rr[4 * q4 + e] = rscale * (yq[e] - pm);
                    }
                }
                const u16x8 r0 = pack_bf16(rr, 0), r1 = pack_bf16(rr, 1);
                Rb[(2 * w) * 64 + ln] = r0;
                Rb[(2 * w + 1) * 64 + ln] = r1;
                float rs = frag_sum(r1, frag_sum(r0, 0.f));
                rs += __shfl_xor(rs, 32);
                if (h == 0) rsum[w * 32 + col] = rs;
            } else {
#pragma unroll
                for (int p = 0; p < kPA; ++p)
                    ra[p] = qa[((size_t)(o0 + p / KPA2) * KPA2 + p % KPA2) * 64 + ln];
            }
            __syncthreads();   // C
            // ---- adjoint Z_i = Q^T R'' for own i, bias removed; A1: W_i; W -> LDS
            {
                float rsall = 0.f;
#pragma unroll
                for (int v = 0; v < TT; ++v) rsall += rsum[v * 32 + col];
                const float zb = 192.f * rsall;
                floatx16 wprev;   // W of the even t of the pair being built
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    floatx16 z;   // started at -192 rsum: the bias of the widened Q cancels
#pragma unroll
                    for (int r = 0; r < 16; ++r) z[r] = -zb;
#pragma unroll 1
                    for (int g0 = 0; g0 < KPA2; g0 += kPA) {
#pragma unroll
                        for (int j = 0; j < kPA; ++j) {
                            const u32x4 qq = ra[j];
                            const int g2 = t * KPA2 + g0 + j + kPA;   // pair whose fragments replace it
                            if (g2 < 4 * KPA2)
                                ra[j] = qa[((size_t)(o0 + g2 / KPA2) * KPA2 + g2 % KPA2) * 64 + ln];
                            z = mma(widen_q(qq.xy), Rb[(2 * (g0 + j)) * 64 + ln], z);
                            z = mma(widen_q(qq.zw), Rb[(2 * (g0 + j) + 1) * 64 + ln], z);
                        }
                    }
                    floatx16 wt = mma(cn(0), pack_bf16(z, 0), floatx16{});
                    wt = mma(cn(1), pack_bf16(z, 1), wt);
                    if (t & 1) {
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            XW1[(rho_row(r, h) * 256 + share) * 2 + (t >> 1)] = cvt2(wprev[r], wt[r]);
                    } else {
                        wprev = wt;
                    }
                }
            }
            __syncthreads();   // D
            // ---- A2 from v, then threshold and momentum
            const float bk = beta[k];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int l = o0 + t;
                floatx16 u = mma(cn(0), XW[(2 * l) * 64 + ln], vv[t]);
                u = mma(cn(1), XW[(2 * l + 1) * 64 + ln], u);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float sn = u[r] - __builtin_amdgcn_fmed3f(u[r], -tau, tau);
                    vv[t][r] = fmaf(bk, sn - sp[t][r], sn);
                    sp[t][r] = sn;
                }
            }
        }
        // ---- write s_T: coefficient (k, l) at 32 k + l
        if (col < nblk) {
            float* dst = tl.s + (size_t)col * kQN;
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int r = 0; r < 16; ++r) dst[32 * rho_row(r, h) + o0 + t] = sp[t][r];
        }
    }
}

template <int MP, int PF, int PA>
static void launch_q8(const FusedTile* tiles, const int* qoff, const int* queue, int* counters,
                      int grid, hipStream_t st) {
    constexpr size_t lds = 131072 + (size_t)(MP / 16) * 1024 + 2 * 8 * 32 * 4 + 4 * 1024;
    static_assert(lds + 64 <= 160 * 1024, "LDS of the workgroup exceeds a CU");
    ensure_lds_limit<&fista_q8_kernel<MP, PF, PA>>(lds);
    fista_q8_kernel<MP, PF, PA><<<dim3(grid), dim3(512), lds, st>>>(tiles, qoff, queue, counters);
    CSV_HIP(hipGetLastError());
}

void launch_fista_q8_m256(const FusedTile* tiles, const int* qoff, const int* queue,
                          int* counters, int grid, hipStream_t st) {
    launch_q8<256, 2, 2>(tiles, qoff, queue, counters, grid, st);
}

}  // namespace csv
