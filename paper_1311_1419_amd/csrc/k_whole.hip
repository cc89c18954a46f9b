// Whole-frame measurement (eq. (1) read literally): each CS frame's residual
// r_t = F_t - F^_key (eqs. (2)-(3)) is one vector of n = W H pixels, measured
// by the stream's M x n integer matrix Q, y~_t = Q r_t, and quantised with
// the block-floating-point rule, the frame being one block.  Q comes from the
// counter generator entry by entry (Q[i][j] = popcount of word (i n + j) mod 4
// of the Philox block at counter ((i n + j) / 4, n, 0, 0)) inside the kernel:
// it is never stored.  The work is integer ALU bound: one Philox4x64-10 block
// per four entries of Q, each entry multiplied into every CS frame.
#include "internal.h"
#include "philox.h"
#include "tv_step.h"

namespace csv {

constexpr int kWRows = 64;     // rows of Q per workgroup (four threads per row)
constexpr int kWCols = 512;    // columns (pixels) per workgroup
constexpr int kWMaxF = 31;     // CS frames per GOP

// Grid (ceil(M / 64), ceil(n / 512)).  The residual of the workgroup's 512
// pixels of every CS frame is staged in LDS as int16; thread (row i, part p)
// generates the Q entries of columns 4 p + 16 c and accumulates q r over them
// in int32 (each partial is below 2^22); the four parts of a row are summed
// with lane shuffles and added to y (int64) with one atomic per row and frame.
__global__ __launch_bounds__(256) void whole_measure_kernel(const uint8_t* __restrict__ frames,
                                                            int n_frames, size_t frame_stride,
                                                            const uint8_t* __restrict__ key, int n,
                                                            int M, uint64_t k0, uint64_t k1,
                                                            unsigned long long* __restrict__ y) {
    __shared__ __attribute__((aligned(16))) int16_t rs[kWMaxF][kWCols];
    const int tid = threadIdx.x;
    const int row0 = blockIdx.x * kWRows, col0 = blockIdx.y * kWCols;
    const int ncols = min(kWCols, n - col0);   // a multiple of 8 (n % 8 == 0)
    for (int e = tid; e < n_frames * (kWCols / 8); e += 256) {
        const int t = e / (kWCols / 8), c8 = (e - t * (kWCols / 8)) * 8;
        short v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (c8 < ncols) {
            const uint2 f = *reinterpret_cast<const uint2*>(frames + t * frame_stride + col0 + c8);
            const uint2 k = *reinterpret_cast<const uint2*>(key + col0 + c8);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                v[b] = (short)((int)((f.x >> (8 * b)) & 0xffu) - (int)((k.x >> (8 * b)) & 0xffu));
                v[4 + b] = (short)((int)((f.y >> (8 * b)) & 0xffu) - (int)((k.y >> (8 * b)) & 0xffu));
            }
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) rs[t][c8 + b] = v[b];
    }
    __syncthreads();
    const int i = row0 + (tid >> 2), part = tid & 3;
    int acc[kWMaxF];
#pragma unroll
    for (int t = 0; t < kWMaxF; ++t) acc[t] = 0;
    if (i < M) {
        for (int k = 4 * part; k < ncols; k += 16) {
            uint64_t c0 = ((uint64_t)i * (uint64_t)n + (uint64_t)(col0 + k)) >> 2;
            uint64_t c1 = (uint64_t)n, c2 = 0, c3 = 0;
            philox4x64_10(c0, c1, c2, c3, k0, k1);
            const int q0 = __popcll(c0) - 32, q1 = __popcll(c1) - 32;
            const int q2 = __popcll(c2) - 32, q3 = __popcll(c3) - 32;
#pragma unroll
            for (int t = 0; t < kWMaxF; ++t) {
                if (t < n_frames)
                    acc[t] += q0 * rs[t][k] + q1 * rs[t][k + 1] + q2 * rs[t][k + 2] +
                              q3 * rs[t][k + 3];
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kWMaxF; ++t) {
        int v = acc[t];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        if (t < n_frames && part == 0 && i < M)
            atomicAdd(&y[(size_t)t * M + i], (unsigned long long)(long long)v);
    }
}

// One workgroup per frame: m = max |y~|, e = min{e >= 0 : (m + h(e)) >> e <=
// 127} with h(0) = 0, h(e) = 2^(e-1); code = sgn(y~) ((|y~| + h(e)) >> e).
__global__ __launch_bounds__(256) void whole_quantise_kernel(const long long* __restrict__ y, int M,
                                                             int8_t* __restrict__ codes,
                                                             uint8_t* __restrict__ exps,
                                                             int32_t* __restrict__ y32) {
    __shared__ long long red[256];
    const int f = blockIdx.x, tid = threadIdx.x;
    const long long* row = y + (size_t)f * M;
    long long mx = 0;
    for (int m = tid; m < M; m += 256) mx = max(mx, llabs(row[m]));
    red[tid] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = max(red[tid], red[tid + s]);
        __syncthreads();
    }
    mx = red[0];
    int e = 0;
    while (((mx + (e ? (1ll << (e - 1)) : 0ll)) >> e) > 127) ++e;
    const long long h = e ? (1ll << (e - 1)) : 0ll;
    for (int m = tid; m < M; m += 256) {
        const long long v = row[m];
        const long long a = (llabs(v) + h) >> e;
        codes[(size_t)f * M + m] = (int8_t)(v < 0 ? -a : a);
        if (y32) y32[(size_t)f * M + m] = (int32_t)v;
    }
    if (tid == 0) exps[f] = (uint8_t)e;
}

void launch_whole_measure(const Shape& s, const uint8_t* frames, int n_frames, size_t frame_stride,
                          const uint8_t* key, long long* y, hipStream_t st) {
    if (n_frames <= 0) return;
    CSV_REQUIRE(n_frames <= kWMaxF, CSV_EUNSUPPORTED, "whole-frame measurement: GOP above 32");
    CSV_REQUIRE(s.n % 8 == 0 && frame_stride % 8 == 0 &&
                    ((reinterpret_cast<uintptr_t>(frames) | reinterpret_cast<uintptr_t>(key)) % 8) == 0,
                CSV_EINVAL, "frame buffers must be 8-byte aligned");
    launch_fill_u64(reinterpret_cast<unsigned long long*>(y), 0ull, n_frames * s.M, st);
    const dim3 grid((unsigned)ceil_div(s.M, kWRows), (unsigned)ceil_div(s.n, kWCols));
    whole_measure_kernel<<<grid, dim3(256), 0, st>>>(frames, n_frames, frame_stride, key, s.n, s.M,
                                                     s.seed, (uint64_t)s.sid,
                                                     reinterpret_cast<unsigned long long*>(y));
    CSV_HIP(hipGetLastError());
}

void launch_whole_quantise(const long long* y, int M, int n_frames, int8_t* codes, uint8_t* exps,
                           int32_t* y32, hipStream_t st) {
    if (n_frames <= 0) return;
    whole_quantise_kernel<<<dim3(n_frames), dim3(256), 0, st>>>(y, M, codes, exps, y32);
    CSV_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- decode
// Whole-frame recovery (eq. (1) with the TV solver of k_tv.hip, each CS frame
// one W x H image): Phi = s_Phi Q with Q (M x n int8) resident; F frames.

// Both products stage a 512-column chunk of the dense operand (x or r) in
// LDS, column c at lds_col(c) in rows of 640 floats: the eight 16-float
// pieces that one load instruction of a wave reads (lanes 16 part + 128 u
// for part 0..7) then start in eight different groups of four banks, free of
// conflicts.  Each thread takes R rows of Q (R pixel rows of Q^T), so every
// value read from LDS feeds R multiply-adds; FM bounds the frames of a GOP
// (F <= FM), fixing the accumulator count.
constexpr int kFwdCols = 512;   // pixels per forward workgroup (one sum chunk)
constexpr int kAdjRows = 512;   // rows of Q^T staged per adjoint step
constexpr int kLdsRow = 640;    // floats per staged row (512 columns, swizzled)
constexpr int kNT = 256;        // threads per product workgroup
static_assert(kNT % (kFwdCols / 4) == 0 && kAdjRows % kNT == 0,
              "the staging loops need whole steps of the workgroup");

__device__ inline int lds_col(int c) { return (c >> 7) * 160 + (c & 127) + 4 * ((c >> 4) & 7); }

// a / d for 0 <= a < 2^21 and 0 < d (pixel indices of the whole-frame
// decoder, whose exact int32 Gram matrix bounds W H below 2^21): the float
// estimate a * (1 / d) is within one of the quotient; an exact integer
// correction follows.
__device__ inline int div_small(int a, int d, float inv_d) {
    int qd = (int)((float)a * inv_d);
    qd -= qd * d > a ? 1 : 0;
    qd += (qd + 1) * d <= a ? 1 : 0;
    return qd;
}

// Unpack 16 signed bytes to floats (exact).
__device__ inline void unpack16(const int4& qq, float* qv) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int wd = e == 0 ? qq.x : e == 1 ? qq.y : e == 2 ? qq.z : qq.w;
#pragma unroll
        for (int b = 0; b < 4; ++b) qv[4 * e + b] = (float)(int8_t)((wd >> (8 * b)) & 0xff);
    }
}

// acc[rho][f] += sum of the 16 products of piece (qv[rho], staged row f at
// physical column base) over rho < R, f < F.
template <int FM, int R>
__device__ inline void piece_fma(const float (&qv)[R][16], const float* __restrict__ st, int base,
                                 int F, float (&acc)[R][FM]) {
#pragma unroll
    for (int f = 0; f < FM; ++f) {
        if (f < F) {
            const float4* sf = reinterpret_cast<const float4*>(st + f * kLdsRow + base);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float4 v = sf[e];
#pragma unroll
                for (int rho = 0; rho < R; ++rho) {
                    acc[rho][f] = fmaf(qv[rho][4 * e], v.x, acc[rho][f]);
                    acc[rho][f] = fmaf(qv[rho][4 * e + 1], v.y, acc[rho][f]);
                    acc[rho][f] = fmaf(qv[rho][4 * e + 2], v.z, acc[rho][f]);
                    acc[rho][f] = fmaf(qv[rho][4 * e + 3], v.w, acc[rho][f]);
                }
            }
        }
    }
}

// Forward product with the dual step.  Partials P[k][g][f][m] = sum over
// the pixels p of chunk k (512 pixels) of Q_g[m][p] x[g][f][p] for the GOPs g
// of a batch (one Q each, same shape), added in chunk order by
// whole_fwd_reduce_kernel: the sums depend only on the shapes.  Grid
// (ceil(M / (NT / 8) R), ceil(n / 512), GOPs), NT threads: eight lanes share
// a row of Q (rows m0 + (NT / 8) rho), each reading 16 bytes at 128 u +
// 16 part (a wave reads whole 128-byte lines); all of a thread's pieces are
// requested before the chunk of x is staged.  The last chunk may be shorter
// (a multiple of 64, as n is).  With tv set, the workgroups of a chunk also
// take the dual step of its pixels (each row tile a slice): it reads x only
// and writes nu, w, P, which the adjoint launch reads.
template <int FM, int R, int NT>
__global__ __launch_bounds__(NT) void whole_fwd_kernel(WholeQ qs, const float* __restrict__ xall,
                                                       int F, int H, int W, int M,
                                                       float* __restrict__ part_out, WholeTv tv) {
    constexpr int RS = NT / 8;   // row stride between a thread's rows
    extern __shared__ float xs[];   // F x kLdsRow
    const int n = H * W;
    const int tid = threadIdx.x, col0 = blockIdx.y * kFwdCols, g = blockIdx.z;
    const int ncols = min(kFwdCols, n - col0);
    const int8_t* __restrict__ q = qs.q[g];
    const float* __restrict__ x = xall + (size_t)g * F * n;
    const int part = tid & 7, mb = blockIdx.x * (RS * R) + (tid >> 3);
    int4 qq[R][kFwdCols / 128];
#pragma unroll
    for (int rho = 0; rho < R; ++rho) {
        const int m = mb + RS * rho;
#pragma unroll
        for (int u = 0; u < kFwdCols / 128; ++u) {
            const int c = 16 * part + 128 * u;
            qq[rho][u] = m < M && c < ncols
                             ? *reinterpret_cast<const int4*>(q + (size_t)m * n + col0 + c)
                             : make_int4(0, 0, 0, 0);
        }
    }
    {
        // F x 128 float4 over NT threads (FS frames per step), loaded from
        // clamped in-range addresses so that all are in flight
        constexpr int FS = NT / (kFwdCols / 4);
        const int c4 = (tid % (kFwdCols / 4)) * 4, fr = tid / (kFwdCols / 4);
        const int cc = c4 < ncols ? c4 : 0;
        float4 xv[(FM + FS - 1) / FS];
#pragma unroll
        for (int s4 = 0; s4 < (FM + FS - 1) / FS; ++s4) {
            const int f = min(FS * s4 + fr, F - 1);
            xv[s4] = FS * s4 < F ? *reinterpret_cast<const float4*>(x + (size_t)f * n + col0 + cc)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int s4 = 0; s4 < (FM + FS - 1) / FS; ++s4)
            if (FS * s4 + fr < F && c4 < ncols)
                *reinterpret_cast<float4*>(xs + (FS * s4 + fr) * kLdsRow + lds_col(c4)) = xv[s4];
    }
    __syncthreads();
    float acc[R][FM];
#pragma unroll
    for (int rho = 0; rho < R; ++rho)
#pragma unroll
        for (int f = 0; f < FM; ++f) acc[rho][f] = 0.f;
#pragma unroll
    for (int u = 0; u < kFwdCols / 128; ++u) {
        const int c = 16 * part + 128 * u;
        if (c >= ncols) break;
        float qv[R][16];
#pragma unroll
        for (int rho = 0; rho < R; ++rho) unpack16(qq[rho][u], qv[rho]);
        piece_fma<FM, R>(qv, xs, lds_col(c), F, acc);
    }
    float* out = part_out + ((size_t)blockIdx.y * gridDim.z + g) * F * M;
#pragma unroll
    for (int rho = 0; rho < R; ++rho) {
        const int m = mb + RS * rho;
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            float v = acc[rho][f];
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            // every lane of the row holds the sum: lane f % 8 stores frame f
            if (f < F && (f & 7) == part && m < M) out[(size_t)f * M + m] = v;
        }
    }
    if (tv.nuh) {
        const int tiles = gridDim.x, t = blockIdx.x;
        const int lo = ncols * t / tiles, hi = ncols * (t + 1) / tiles, cnt = hi - lo;
        const float invc = 1.f / (float)cnt, invW = 1.f / (float)W;
        for (int e = tid; e < F * cnt; e += NT) {
            const int f = div_small(e, cnt, invc), k = col0 + lo + (e - f * cnt);
            const int i = div_small(k, W, invW), j = k - i * W;
            const int b = g * F + f;
            tv_dual_at(xall + (size_t)b * n, k, i, j, H, W, (size_t)b * n + k, tv.lam[b], tv.nuh,
                       tv.nuv, tv.wh, tv.wv, tv.ph, tv.pv);
        }
    }
}

// r[i] = s_Phi sum_k P[k][i] - y^[i] over i = (g, f, m) (chunks in order).
__global__ __launch_bounds__(256) void whole_fwd_reduce_kernel(const float* __restrict__ part,
                                                               int nk, int count, float s_phi,
                                                               const float* __restrict__ y,
                                                               float* __restrict__ r) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    float v = 0.f;
#pragma unroll 8
    for (int k = 0; k < nk; ++k) v += part[(size_t)k * count + idx];
    r[idx] = fmaf(s_phi, v, -y[idx]);
}

// Adjoint product with the primal step.  g[g][f][p] = s_Phi sum_m Q_g[m][p]
// r[g][f][m], read from the transposed copy Q^T (n x Mp, rows zero-padded):
// grid (ceil(n / (NT / 8) R), GOPs), NT threads, eight lanes per pixel row
// (rows p0 + (NT / 8) rho) reading 16 bytes each at 128 u + 16 part, r staged in
// LDS 512 rows at a time after the thread's pieces of Q^T are requested,
// the eight lanes meeting by lane shuffles (fixed order).  With tv set the
// gradient never leaves the registers: x <- x - alpha (g + D^T P) at once
// (P from the dual step of the forward launch); else g is written to gout.
template <int FM, int R, int NT>
__global__ __launch_bounds__(NT) void whole_adj_kernel(WholeQ qts, const float* __restrict__ rall,
                                                       int F, int H, int W, int M, int Mp,
                                                       float s_phi, float* __restrict__ gout,
                                                       WholeTv tv) {
    constexpr int RS = NT / 8;   // pixel-row stride between a thread's rows
    extern __shared__ float rs[];   // F x kLdsRow
    const int n = H * W;
    const int tid = threadIdx.x, g = blockIdx.y, part = tid & 7;
    const int pb = blockIdx.x * (RS * R) + (tid >> 3);
    const float invW = 1.f / (float)W;
    const int8_t* __restrict__ qt = qts.q[g];
    const float* __restrict__ r = rall + (size_t)g * F * M;
    float acc[R][FM];
#pragma unroll
    for (int rho = 0; rho < R; ++rho)
#pragma unroll
        for (int f = 0; f < FM; ++f) acc[rho][f] = 0.f;
    for (int m0 = 0; m0 < Mp; m0 += kAdjRows) {
        const int mch = min(kAdjRows, Mp - m0);   // a multiple of 32
        int4 qq[R][kAdjRows / 128];
#pragma unroll
        for (int rho = 0; rho < R; ++rho) {
            const int p = pb + RS * rho;
#pragma unroll
            for (int u = 0; u < kAdjRows / 128; ++u) {
                const int c = 16 * part + 128 * u;
                qq[rho][u] = p < n && c < mch
                                 ? *reinterpret_cast<const int4*>(qt + (size_t)p * Mp + m0 + c)
                                 : make_int4(0, 0, 0, 0);
            }
        }
        if (m0) __syncthreads();
#pragma unroll
        for (int h = 0; h < kAdjRows / NT; ++h) {
            float rv[FM];   // thread tid stages rows m0 + tid + NT h of every frame
            const int mm = tid + NT * h;
            const int mr = m0 + mm < M ? m0 + mm : M - 1;
#pragma unroll
            for (int f = 0; f < FM; ++f) rv[f] = f < F ? r[(size_t)f * M + mr] : 0.f;
#pragma unroll
            for (int f = 0; f < FM; ++f)
                if (f < F && mm < mch) rs[f * kLdsRow + lds_col(mm)] = m0 + mm < M ? rv[f] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kAdjRows / 128; ++u) {
            const int c = 16 * part + 128 * u;
            if (c >= mch) break;
            float qv[R][16];
#pragma unroll
            for (int rho = 0; rho < R; ++rho) unpack16(qq[rho][u], qv[rho]);
            piece_fma<FM, R>(qv, rs, lds_col(c), F, acc);
        }
    }
#pragma unroll
    for (int rho = 0; rho < R; ++rho) {
        const int p = pb + RS * rho;
        const int i = div_small(p, W, invW), j = p - i * W;
        float sums[FM];
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            float v = acc[rho][f];
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            sums[f] = v;   // every lane of the row holds every frame's sum
        }
        // lane part finishes frames part, part + 8, ...
#pragma unroll
        for (int f0 = 0; f0 < FM; f0 += 8) {
            const int f = f0 + part;
            float v = 0.f;
#pragma unroll
            for (int ff = 0; ff < 8 && f0 + ff < FM; ++ff) v = part == ff ? sums[f0 + ff] : v;
            if (f < F && p < n) {
                const int b = g * F + f;
                const float gv = s_phi * v;
                if (!tv.nuh) {
                    gout[(size_t)b * n + p] = gv;
                } else {
                    const float dt = tv_dtp_at(tv.ph + (size_t)b * n, tv.pv + (size_t)b * n, p, i,
                                               j, H, W);
                    tv.x[(size_t)b * n + p] -= tv.alpha[b] * (gv + dt);
                }
            }
        }
    }
}

// Q^T (n x Mp) from Q (Mp x n): 32 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void transpose_q_kernel(const int8_t* __restrict__ q, int Mp,
                                                          int n, int8_t* __restrict__ qt) {
    __shared__ int8_t t[32][65];
    const int m0 = blockIdx.y * 32, p0 = blockIdx.x * 64, tid = threadIdx.x;
    for (int e = tid; e < 32 * 64; e += 256) {
        const int r = e / 64, c = e % 64;
        t[r][c] = q[(size_t)(m0 + r) * n + p0 + c];
    }
    __syncthreads();
    for (int e = tid; e < 32 * 64; e += 256) {
        const int c = e / 32, r = e % 32;
        qt[(size_t)(p0 + c) * Mp + m0 + r] = t[r][c];
    }
}

__global__ void whole_alpha_kernel(WholeLip ls, const float* __restrict__ lam, int F, int nimg,
                                   float* __restrict__ alpha) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nimg) alpha[b] = tv_alpha(ls.lip[b / F][0], tv_beta(lam[b]));
}

// Decoded CS frames: out[f][p] = clip(round-half-even(key[p] + x[f][p])).
__global__ void whole_place_kernel(const float* __restrict__ x, const uint8_t* __restrict__ key,
                                   int F, int n, uint8_t* __restrict__ out,
                                   float* __restrict__ out_f32) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)F * n) return;
    const int p = (int)(idx % n);
    const float f = (float)key[p] + x[idx];
    if (out_f32) out_f32[idx] = f;
    out[idx] = (uint8_t)fminf(fmaxf(rintf(f), 0.f), 255.f);
}

// FP64 check, pass 1: per row m and frame f, d = s_Phi Q[m] . x[f] - y^[f][m]
// with y^ = s_Phi c 2^e exact; rr = d^2, yy = y^2 (one wave per row).
__global__ __launch_bounds__(256) void whole_obj_rows_kernel(const int8_t* __restrict__ q,
                                                             const float* __restrict__ x, int F,
                                                             int n, int M, double s_phi,
                                                             const int8_t* __restrict__ codes,
                                                             const uint8_t* __restrict__ exps,
                                                             double* __restrict__ rr,
                                                             double* __restrict__ yy) {
    const int m = blockIdx.x * 4 + (threadIdx.x >> 6), ln = threadIdx.x & 63;
    if (m >= M) return;
    const int8_t* qr = q + (size_t)m * n;
    for (int f = 0; f < F; ++f) {
        double acc = 0.0;
        for (int p = ln; p < n; p += 64) acc += (double)qr[p] * (double)x[(size_t)f * n + p];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (ln == 0) {
            const double yh = s_phi * ldexp((double)codes[(size_t)f * M + m], (int)exps[f]);
            const double d = s_phi * acc - yh;
            rr[(size_t)f * M + m] = d * d;
            yy[(size_t)f * M + m] = yh * yh;
        }
    }
}

// Pass 2, one workgroup per frame, fixed summation order: obj = 1/2 sum rr +
// lam TV(x) (FP64), rel = sqrt(sum rr / sum yy).
__global__ __launch_bounds__(256) void whole_obj_final_kernel(const double* __restrict__ rr,
                                                              const double* __restrict__ yy,
                                                              const float* __restrict__ x,
                                                              const float* __restrict__ lam, int M,
                                                              int H, int W,
                                                              double* __restrict__ obj) {
    __shared__ double red[3][256];
    const int f = blockIdx.x, tid = threadIdx.x, n = H * W;
    double a = 0.0, b = 0.0, t = 0.0;
    for (int m = tid; m < M; m += 256) {
        a += rr[(size_t)f * M + m];
        b += yy[(size_t)f * M + m];
    }
    const float* xf = x + (size_t)f * n;
    for (int k = tid; k < n; k += 256) {
        const int i = k / W, j = k - i * W;
        const double v = xf[k];
        const double dh = j + 1 < W ? (double)xf[k + 1] - v : 0.0;
        const double dv = i + 1 < H ? (double)xf[k + W] - v : 0.0;
        t += sqrt(dh * dh + dv * dv);
    }
    red[0][tid] = a;
    red[1][tid] = b;
    red[2][tid] = t;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            red[0][tid] += red[0][tid + s];
            red[1][tid] += red[1][tid + s];
            red[2][tid] += red[2][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        obj[(size_t)f * 2 + 0] = 0.5 * red[0][0] + (double)lam[f] * red[2][0];
        obj[(size_t)f * 2 + 1] = red[1][0] > 0.0 ? sqrt(red[0][0]) / sqrt(red[1][0]) : 0.0;
    }
}

int whole_fwd_parts(int n) { return ceil_div(n, kFwdCols); }

void launch_whole_fwd(const WholeQ& qs, int ngop, const float* x, int F, int H, int W, int M,
                      float s_phi, const float* y, float* part, float* r, const WholeTv& tv,
                      hipStream_t st) {
    const int n = H * W;
    if (F <= 0 || ngop <= 0) return;
    CSV_REQUIRE(F <= kWMaxF && n % 64 == 0 && ngop <= kWholeBatch, CSV_EUNSUPPORTED,
                "whole-frame product shape");
    const int nk = whole_fwd_parts(n);
    const size_t lds = (size_t)F * kLdsRow * sizeof(float);
    auto go = [&](auto kern, int R) {
        kern<<<dim3(ceil_div(M, kNT / 8 * R), nk, ngop), dim3(kNT), lds, st>>>(qs, x, F, H, W, M,
                                                                              part, tv);
    };
    if (F <= 4)
        go(whole_fwd_kernel<4, 2, kNT>, 2);
    else if (F <= 8)
        go(whole_fwd_kernel<8, 2, kNT>, 2);
    else if (F <= 16)
        go(whole_fwd_kernel<16, 1, kNT>, 1);
    else
        go(whole_fwd_kernel<32, 1, kNT>, 1);
    CSV_HIP(hipGetLastError());
    const int count = ngop * F * M;
    whole_fwd_reduce_kernel<<<dim3(ceil_div(count, 256)), dim3(256), 0, st>>>(part, nk, count,
                                                                             s_phi, y, r);
    CSV_HIP(hipGetLastError());
}

void launch_whole_adj(const WholeQ& qts, int ngop, const float* r, int F, int H, int W, int M,
                      int Mp, float s_phi, float* gout, const WholeTv& tv, hipStream_t st) {
    const int n = H * W;
    if (F <= 0 || ngop <= 0) return;
    CSV_REQUIRE(F <= kWMaxF && n % 64 == 0 && Mp % 32 == 0 && Mp >= M && ngop <= kWholeBatch,
                CSV_EUNSUPPORTED, "whole-frame product shape");
    const size_t lds = (size_t)F * kLdsRow * sizeof(float);
    auto go = [&](auto kern, int R) {
        kern<<<dim3(ceil_div(n, kNT / 8 * R), ngop), dim3(kNT), lds, st>>>(qts, r, F, H, W, M, Mp,
                                                                          s_phi, gout, tv);
    };
    if (F <= 4)
        go(whole_adj_kernel<4, 4, kNT>, 4);
    else if (F <= 8)
        go(whole_adj_kernel<8, 2, kNT>, 2);
    else if (F <= 16)
        go(whole_adj_kernel<16, 1, kNT>, 1);
    else
        go(whole_adj_kernel<32, 1, kNT>, 1);
    CSV_HIP(hipGetLastError());
}

void launch_transpose_q(const int8_t* q, int Mp, int n, int8_t* qt, hipStream_t st) {
    CSV_REQUIRE(Mp % 32 == 0 && n % 64 == 0, CSV_EUNSUPPORTED, "transpose shape");
    transpose_q_kernel<<<dim3(n / 64, Mp / 32), dim3(256), 0, st>>>(q, Mp, n, qt);
    CSV_HIP(hipGetLastError());
}

void launch_whole_alpha(const WholeLip& ls, const float* lam, int F, int ngop, float* alpha,
                        hipStream_t st) {
    if (ngop <= 0 || F <= 0) return;
    CSV_REQUIRE(ngop <= kWholeBatch, CSV_EINVAL, "whole-frame batch too large");
    whole_alpha_kernel<<<dim3(ceil_div(ngop * F, 256)), dim3(256), 0, st>>>(ls, lam, F, ngop * F,
                                                                           alpha);
    CSV_HIP(hipGetLastError());
}

void launch_whole_place(const float* x, const uint8_t* key, int F, int n, uint8_t* out,
                        float* out_f32, hipStream_t st) {
    const size_t t = (size_t)F * n;
    if (!t) return;
    whole_place_kernel<<<dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st>>>(x, key, F, n, out,
                                                                               out_f32);
    CSV_HIP(hipGetLastError());
}

void launch_whole_objective(const int8_t* q, const float* x, int F, int H, int W, int M,
                            double s_phi, const int8_t* codes, const uint8_t* exps,
                            const float* lam, double* rr, double* yy, double* obj,
                            hipStream_t st) {
    if (F <= 0) return;
    whole_obj_rows_kernel<<<dim3(ceil_div(M, 4)), dim3(256), 0, st>>>(q, x, F, H * W, M, s_phi,
                                                                     codes, exps, rr, yy);
    CSV_HIP(hipGetLastError());
    whole_obj_final_kernel<<<dim3(F), dim3(256), 0, st>>>(rr, yy, x, lam, M, H, W, obj);
    CSV_HIP(hipGetLastError());
}

}  // namespace csv
