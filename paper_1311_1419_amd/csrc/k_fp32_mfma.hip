// Plain FP32 recovery on the FP32 matrix cores: the two products of every
// iteration (forward R = V A^T - y^, adjoint G = R A) as tiled GEMMs on
// v_mfma_f32_32x32x2_f32 (FP32 products, FP32 accumulation), for a batch of
// GOPs of one shape that share every launch (grid.z = GOP, each GOP's
// operator and arrays passed by value); the threshold and momentum step
// runs in the adjoint's epilogue.  The sums run in a fixed order: results depend only on the
// shapes, and a GOP decodes identically alone or in a batch.
#include "internal.h"
#include "mfma.h"

namespace csv {

// Workgroup tile 128 x TN of C (TN = 128, or 64 for narrow outputs), four
// waves in 2 x 2, each 64 x TN/2 (2 x TN/64 accumulator tiles of 32 x 32);
// K in chunks of 16 staged in LDS (X as [k][row], B as [k][col], both padded
// by 4 floats per row), double buffered, the next chunk's global loads in
// flight during the MFMAs.
constexpr int kGM = 128, kGK = 16, kGP = kGM + 4;

// Epilogues of the adjoint product: store G, the FISTA step on (S, V), or
// the monotone variant's prox step z = soft(V - G / L, lam / L) into Z.
enum { kEpiStore = 0, kEpiFista = 1, kEpiZStep = 2 };

// C = X B for GOP g = blockIdx.z, rows of X are blocks (b < nblk):
//   FWD: X = V_g (nblk x K, K = n), B[k][c] = A_g[c][k] (c over Mp);
//        C = R_g (nblk x Mp): acc - y^_g for c < M (acc itself when y^_g
//        is NULL), 0 for M <= c < Mp.
//   ADJ: X = R_g (nblk x K, K = Mp), B[k][c] = A_g[k][c] (c over n);
//        C = G_g (nblk x n), or with EPI the FISTA step of iteration k on
//        (S_g, V_g), or the prox step into Z_g, from each G entry, which is
//        then not stored.
template <bool FWD, int TN, int EPI = kEpiStore>
__global__ __launch_bounds__(256) void f32_gemm_kernel(F32Batch bt, int N, int K, int M,
                                                      const float* __restrict__ beta = nullptr,
                                                      int kit = 0) {
    static_assert(!(FWD && EPI != kEpiStore), "the step follows the adjoint product");
    constexpr int NJ = TN / 64;     // accumulator tiles per wave along the columns
    constexpr int NB = TN / 64;     // float4 of B staged per thread per chunk
    const F32Job& jb = bt.j[blockIdx.z];
    const int nblk = jb.nblk;
    const int r0 = blockIdx.y * kGM, c0 = blockIdx.x * TN;
    if (r0 >= nblk) return;   // the whole workgroup: this GOP has fewer blocks
    const float* __restrict__ X = FWD ? jb.V : jb.R;
    const float* __restrict__ W = jb.op;   // Mp x n, row-major
    const int ldw = FWD ? K : N;
    __shared__ float Xs[2][kGK][kGP];
    __shared__ float Bs[2][kGK][TN + 4];
    const int tid = threadIdx.x, w = tid >> 6, ln = tid & 63;
    const int wr = (w >> 1) * 64, wc = (w & 1) * (TN / 2);

    // per-thread staging: two float4 of X (rows e / 4, k (e % 4) 4) and NB
    // of B (FWD: cols e / 4, k (e % 4) 4; ADJ: k e / (TN / 4), cols
    // (e % (TN / 4)) 4)
    float4 xr[2], br[NB];
    auto load = [&](int k0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = tid + 256 * h;
            const int row = e >> 2, kq = (e & 3) * 4;
            xr[h] = r0 + row < nblk
                        ? *reinterpret_cast<const float4*>(X + (size_t)(r0 + row) * K + k0 + kq)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int h = 0; h < NB; ++h) {
            const int e = tid + 256 * h;
            if (FWD) {
                const int col = e >> 2, kq = (e & 3) * 4;
                const float* src = W + (size_t)(c0 + col) * ldw + k0 + kq;
                br[h] = c0 + col < N ? *reinterpret_cast<const float4*>(src)
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
            } else {
                const int kr = e / (TN / 4), cq = (e % (TN / 4)) * 4;
                const float* src = W + (size_t)(k0 + kr) * ldw + c0 + cq;
                br[h] = c0 + cq < N ? *reinterpret_cast<const float4*>(src)
                                    : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = tid + 256 * h;
            const int row = e >> 2, kq = (e & 3) * 4;
            Xs[buf][kq + 0][row] = xr[h].x;
            Xs[buf][kq + 1][row] = xr[h].y;
            Xs[buf][kq + 2][row] = xr[h].z;
            Xs[buf][kq + 3][row] = xr[h].w;
        }
#pragma unroll
        for (int h = 0; h < NB; ++h) {
            const int e = tid + 256 * h;
            if (FWD) {
                const int col = e >> 2, kq = (e & 3) * 4;
                Bs[buf][kq + 0][col] = br[h].x;
                Bs[buf][kq + 1][col] = br[h].y;
                Bs[buf][kq + 2][col] = br[h].z;
                Bs[buf][kq + 3][col] = br[h].w;
            } else {
                const int kr = e / (TN / 4), cq = (e % (TN / 4)) * 4;
                *reinterpret_cast<float4*>(&Bs[buf][kr][cq]) = br[h];
            }
        }
    };

    floatx16 acc[2][NJ];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = floatx16{};
    const int kh = ln >> 5, lc = ln & 31;
    load(0);
    store(0);
    __syncthreads();
    const int nch = K / kGK;
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) load((ch + 1) * kGK);   // in flight during this chunk's MFMAs
#pragma unroll
        for (int ks = 0; ks < kGK / 2; ++ks) {
            const int kk = 2 * ks + kh;
            const float a0 = Xs[buf][kk][wr + lc], a1 = Xs[buf][kk][wr + 32 + lc];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const float b = Bs[buf][kk][wc + 32 * j + lc];
                acc[0][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b, acc[0][j], 0, 0, 0);
                acc[1][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b, acc[1][j], 0, 0, 0);
            }
        }
        if (ch + 1 < nch) store(buf ^ 1);   // the other buffer: last read before the
        __syncthreads();                    // previous barrier
    }
    // accumulator (lane l, register r) = C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
    if constexpr (EPI != kEpiStore) {
        // u = v - g / L; s_k = soft(u, lam / L); v = s_k + beta_k (s_k - s_{k-1})
        // (monotone variant: z_k = soft(u, lam / L) only)
        const float inv_l = (float)(1.0 / jb.lip[0]);
        const float bk = EPI == kEpiFista ? beta[kit] : 0.f;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = r0 + wr + 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
                if (row >= nblk) continue;
                const float tau = jb.lam[row] * inv_l;
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const int col = c0 + wc + 32 * j + lc;
                    if (col < N) {
                        const size_t o = (size_t)row * N + col;
                        const float u = fmaf(-acc[i][j][r], inv_l, jb.V[o]);
                        const float sn = fmaxf(u - tau, 0.f) + fminf(u + tau, 0.f);
                        if constexpr (EPI == kEpiZStep) {
                            jb.Z[o] = sn;
                        } else {
                            jb.V[o] = fmaf(bk, sn - jb.S[o], sn);
                            jb.S[o] = sn;
                        }
                    }
                }
            }
    } else {
        float* __restrict__ C = FWD ? jb.R : jb.G;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = r0 + wr + 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
                    const int col = c0 + wc + 32 * j + lc;
                    if (row < nblk && col < N) {
                        float v = acc[i][j][r];
                        if (FWD)
                            v = col < M ? (jb.y ? v - jb.y[(size_t)row * N + col] : v) : 0.f;
                        C[(size_t)row * N + col] = v;
                    }
                }
    }
}

static void check_batch(const F32Batch& bt, int ngop, int n, int Mp) {
    CSV_REQUIRE(ngop >= 1 && ngop <= kF32Batch, CSV_EINVAL, "FP32 batch size");
    CSV_REQUIRE(n % kGK == 0 && Mp % kGK == 0 && n % 4 == 0, CSV_EUNSUPPORTED,
                "FP32 product shape");
    for (int g = 0; g < ngop; ++g)
        CSV_REQUIRE(bt.j[g].nblk >= 0, CSV_EINVAL, "negative block count");
}

static int max_rows(const F32Batch& bt, int ngop) {
    int m = 0;
    for (int g = 0; g < ngop; ++g) m = std::max(m, bt.j[g].nblk);
    return m;
}

void launch_f32_forward(const F32Batch& bt, int ngop, int n, int M, int Mp, hipStream_t st) {
    check_batch(bt, ngop, n, Mp);
    const int rows = max_rows(bt, ngop);
    if (!rows) return;
    if (Mp <= 64)
        f32_gemm_kernel<true, 64><<<dim3(ceil_div(Mp, 64), ceil_div(rows, kGM), ngop), dim3(256), 0,
                                    st>>>(bt, Mp, n, M);
    else
        f32_gemm_kernel<true, 128><<<dim3(ceil_div(Mp, 128), ceil_div(rows, kGM), ngop), dim3(256),
                                     0, st>>>(bt, Mp, n, M);
    CSV_HIP(hipGetLastError());
}

void launch_f32_adjoint(const F32Batch& bt, int ngop, int n, int Mp, hipStream_t st) {
    check_batch(bt, ngop, n, Mp);
    const int rows = max_rows(bt, ngop);
    if (!rows) return;
    f32_gemm_kernel<false, 128><<<dim3(ceil_div(n, 128), ceil_div(rows, kGM), ngop), dim3(256), 0,
                                  st>>>(bt, n, Mp, Mp);
    CSV_HIP(hipGetLastError());
}

void launch_f32_adjoint_prox(const F32Batch& bt, int ngop, int n, int Mp, const float* beta,
                             int k, hipStream_t st) {
    check_batch(bt, ngop, n, Mp);
    CSV_REQUIRE(beta != nullptr && k >= 0, CSV_EINVAL, "FISTA step table");
    const int rows = max_rows(bt, ngop);
    if (!rows) return;
    f32_gemm_kernel<false, 128, kEpiFista><<<dim3(ceil_div(n, 128), ceil_div(rows, kGM), ngop),
                                             dim3(256), 0, st>>>(bt, n, Mp, Mp, beta, k);
    CSV_HIP(hipGetLastError());
}

void launch_f32_adjoint_zstep(const F32Batch& bt, int ngop, int n, int Mp, hipStream_t st) {
    check_batch(bt, ngop, n, Mp);
    for (int g = 0; g < ngop; ++g)
        CSV_REQUIRE(bt.j[g].Z != nullptr, CSV_EINVAL, "monotone FISTA: no z buffer");
    const int rows = max_rows(bt, ngop);
    if (!rows) return;
    f32_gemm_kernel<false, 128, kEpiZStep><<<dim3(ceil_div(n, 128), ceil_div(rows, kGM), ngop),
                                             dim3(256), 0, st>>>(bt, n, Mp, Mp);
    CSV_HIP(hipGetLastError());
}

// ----------------------------------------------------- monotone FISTA steps
// One wave per block (four blocks per workgroup), GOP blockIdx.y.
// Sums in FP64 over lane-strided elements, then a butterfly; lane 0's sum is
// broadcast so that every lane takes the same decision.
__device__ inline double wave_sum_bcast(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return __shfl(v, 0);
}

__global__ __launch_bounds__(256) void mfista_init_kernel(F32Batch bt, int n, int M, int Mp) {
    const F32Job& jb = bt.j[blockIdx.y];
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6), ln = threadIdx.x & 63;
    if (b >= jb.nblk) return;   // whole waves
    double yy = 0.0;
    for (int m = ln; m < Mp; m += 64) {
        const size_t o = (size_t)b * Mp + m;
        const float y = m < M ? jb.y[o] : 0.f;
        yy += (double)y * y;
        jb.R[o] = -y;   // A v_1 - y^ with v_1 = 0
        jb.AS[o] = 0.f;
    }
    for (int i = ln; i < n; i += 64) {
        const size_t o = (size_t)b * n + i;
        jb.S[o] = 0.f;
        jb.V[o] = 0.f;
    }
    yy = wave_sum_bcast(yy);
    if (ln == 0) jb.FS[b] = 0.5 * yy;   // F(s_0 = 0)
}

__global__ __launch_bounds__(256) void mfista_select_kernel(F32Batch bt, int n, int M, int Mp,
                                                           const float* __restrict__ coef,
                                                           int k) {
    const F32Job& jb = bt.j[blockIdx.y];
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6), ln = threadIdx.x & 63;
    if (b >= jb.nblk) return;   // whole waves
    const size_t on = (size_t)b * n, om = (size_t)b * Mp;
    double l1 = 0.0, r2 = 0.0;
    for (int i = ln; i < n; i += 64) l1 += fabs((double)jb.Z[on + i]);
    for (int m = ln; m < M; m += 64) {
        const double d = (double)jb.AZ[om + m] - (double)jb.y[om + m];
        r2 += d * d;
    }
    l1 = wave_sum_bcast(l1);
    r2 = wave_sum_bcast(r2);
    const double fz = 0.5 * r2 + (double)jb.lam[b] * l1;
    const bool take = fz <= jb.FS[b];   // ties keep z_k
    const float c1 = coef[2 * k], c2 = coef[2 * k + 1];
    for (int i = ln; i < n; i += 64) {
        const float so = jb.S[on + i], z = jb.Z[on + i];
        const float sn = take ? z : so;
        jb.V[on + i] = sn + c1 * (z - sn) + c2 * (sn - so);
        jb.S[on + i] = sn;
    }
    for (int m = ln; m < Mp; m += 64) {
        const float ao = jb.AS[om + m], az = jb.AZ[om + m];
        const float an = take ? az : ao;
        const float av = an + c1 * (az - an) + c2 * (an - ao);
        jb.AS[om + m] = an;
        jb.R[om + m] = m < M ? av - jb.y[om + m] : 0.f;
    }
    if (ln == 0 && take) jb.FS[b] = fz;
}

static void check_mfista(const F32Batch& bt, int ngop) {
    CSV_REQUIRE(ngop >= 1 && ngop <= kF32Batch, CSV_EINVAL, "FP32 batch size");
    for (int g = 0; g < ngop; ++g) {
        const F32Job& j = bt.j[g];
        CSV_REQUIRE(j.nblk >= 0 && j.S && j.V && j.R && j.y && j.lam && j.Z && j.AZ && j.AS &&
                        j.FS,
                    CSV_EINVAL, "monotone FISTA: missing buffers");
    }
}

void launch_mfista_init(const F32Batch& bt, int ngop, int n, int M, int Mp, hipStream_t st) {
    check_mfista(bt, ngop);
    const int rows = max_rows(bt, ngop);
    if (!rows) return;
    mfista_init_kernel<<<dim3(ceil_div(rows, 4), ngop), dim3(256), 0, st>>>(bt, n, M, Mp);
    CSV_HIP(hipGetLastError());
}

void launch_mfista_select(const F32Batch& bt, int ngop, int n, int M, int Mp, const float* coef,
                          int k, hipStream_t st) {
    check_mfista(bt, ngop);
    CSV_REQUIRE(coef != nullptr && k >= 0, CSV_EINVAL, "monotone FISTA coefficient table");
    const int rows = max_rows(bt, ngop);
    if (!rows) return;
    mfista_select_kernel<<<dim3(ceil_div(rows, 4), ngop), dim3(256), 0, st>>>(bt, n, M, Mp, coef,
                                                                            k);
    CSV_HIP(hipGetLastError());
}

}  // namespace csv
