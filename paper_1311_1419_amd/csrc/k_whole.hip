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

// Both products split the long sum into fixed chunks, write one partial per
// chunk and add the partials in chunk order in the consumer: the result
// depends only on the shapes, never on scheduling.
constexpr int kFwdRows = 64;    // rows of Q per forward workgroup
constexpr int kFwdCols = 512;   // pixels per forward workgroup (one sum chunk)
constexpr int kAdjCols = 1024;  // pixels per adjoint workgroup (4 per thread)

// Forward partials: P[k][f][m] = sum over the pixels p of chunk k of
// Q[m][p] x[f][p].  Grid (ceil(M / 64), ceil(n / 512)); the chunk of every
// frame is staged in LDS (F x 512 floats; the last chunk may be shorter, a
// multiple of 64 since n is); thread (row tid / 4, part tid % 4) takes 16
// pixels at 64 c + 16 part and the four parts meet by lane shuffles.
__global__ __launch_bounds__(256) void whole_fwd_kernel(const int8_t* __restrict__ q,
                                                        const float* __restrict__ x, int F, int n,
                                                        int M, float* __restrict__ part_out) {
    extern __shared__ float xs[];   // F x kFwdCols
    const int tid = threadIdx.x, col0 = blockIdx.y * kFwdCols;
    const int ncols = min(kFwdCols, n - col0);
    for (int e = tid; e < F * (kFwdCols / 4); e += 256) {
        const int f = e / (kFwdCols / 4), c4 = (e - f * (kFwdCols / 4)) * 4;
        if (c4 < ncols)
            *reinterpret_cast<float4*>(xs + f * kFwdCols + c4) =
                *reinterpret_cast<const float4*>(x + (size_t)f * n + col0 + c4);
    }
    __syncthreads();
    const int m = blockIdx.x * kFwdRows + (tid >> 2), part = tid & 3;
    float acc[kWMaxF];
#pragma unroll
    for (int f = 0; f < kWMaxF; ++f) acc[f] = 0.f;
    if (m < M) {
        const int8_t* qr = q + (size_t)m * n + col0;
#pragma unroll 2
        for (int c = 16 * part; c < ncols; c += 64) {
            const int4 qq = *reinterpret_cast<const int4*>(qr + c);
            float qv[16];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int wd = e == 0 ? qq.x : e == 1 ? qq.y : e == 2 ? qq.z : qq.w;
#pragma unroll
                for (int b = 0; b < 4; ++b) qv[4 * e + b] = (float)(int8_t)((wd >> (8 * b)) & 0xff);
            }
#pragma unroll
            for (int f = 0; f < kWMaxF; ++f) {
                if (f < F) {
                    const float4* xf = reinterpret_cast<const float4*>(xs + f * kFwdCols + c);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float4 xv = xf[e];
                        acc[f] = fmaf(qv[4 * e], xv.x, acc[f]);
                        acc[f] = fmaf(qv[4 * e + 1], xv.y, acc[f]);
                        acc[f] = fmaf(qv[4 * e + 2], xv.z, acc[f]);
                        acc[f] = fmaf(qv[4 * e + 3], xv.w, acc[f]);
                    }
                }
            }
        }
    }
    float* out = part_out + (size_t)blockIdx.y * F * M;
#pragma unroll
    for (int f = 0; f < kWMaxF; ++f) {
        float v = acc[f];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        if (f < F && part == 0 && m < M) out[(size_t)f * M + m] = v;
    }
}

// r[f][m] = s_Phi sum_k P[k][f][m] - y^[f][m] (chunks in order).
__global__ void whole_fwd_reduce_kernel(const float* __restrict__ part, int nk, int F, int M,
                                        float s_phi, const float* __restrict__ y,
                                        float* __restrict__ r) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= F * M) return;
    float v = 0.f;
    for (int k = 0; k < nk; ++k) v += part[(size_t)k * F * M + idx];
    r[idx] = fmaf(s_phi, v, -y[idx]);
}

// Adjoint partials: G[j][f][p] = sum over the rows m of chunk j (mc rows) of
// Q[m][p] r[f][m].  Grid (ceil(n / 1024), ceil(M / mc)); r of the chunk is
// staged in LDS; each thread takes four consecutive pixels (one 32-bit load
// of Q per row, a wave reading 256 contiguous bytes).
__global__ __launch_bounds__(256) void whole_adj_kernel(const int8_t* __restrict__ q,
                                                        const float* __restrict__ r, int F, int n,
                                                        int M, int mc, float* __restrict__ part_out) {
    extern __shared__ float rs[];   // F x mc
    const int tid = threadIdx.x, m0 = blockIdx.y * mc;
    const int mend = min(M, m0 + mc);
    for (int e = tid; e < F * mc; e += 256) {
        const int f = e / mc, mm = e - f * mc;
        rs[e] = m0 + mm < M ? r[(size_t)f * M + m0 + mm] : 0.f;
    }
    __syncthreads();
    const int p = blockIdx.x * kAdjCols + tid * 4;
    if (p >= n) return;   // n % 64 == 0: the four pixels are all in range
    float acc[kWMaxF][4];
#pragma unroll
    for (int f = 0; f < kWMaxF; ++f)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[f][b] = 0.f;
    const int8_t* qc = q + p;
    for (int m = m0; m < mend; ++m) {
        const int wd = *reinterpret_cast<const int*>(qc + (size_t)m * n);
        float qv[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) qv[b] = (float)(int8_t)((wd >> (8 * b)) & 0xff);
        const float* rm = rs + (m - m0);
#pragma unroll
        for (int f = 0; f < kWMaxF; ++f) {
            if (f < F) {
                const float rv = rm[f * mc];
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[f][b] = fmaf(qv[b], rv, acc[f][b]);
            }
        }
    }
    float* out = part_out + (size_t)blockIdx.y * F * n;
#pragma unroll
    for (int f = 0; f < kWMaxF; ++f)
        if (f < F)
            *reinterpret_cast<float4*>(out + (size_t)f * n + p) =
                make_float4(acc[f][0], acc[f][1], acc[f][2], acc[f][3]);
}

// out[i] = scale (part[0][i] + ... + part[nparts-1][i]) (parts in order).
__global__ void sum_parts_kernel(const float* __restrict__ part, int nparts, size_t count,
                                 float scale, float* __restrict__ out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float v = part[i];
    for (int k = 1; k < nparts; ++k) v += part[k * count + i];
    out[i] = scale * v;
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

int whole_adj_rows(int M) { return M <= 2048 ? 64 : 256; }

void launch_whole_fwd(const int8_t* q, const float* x, int F, int n, int M, float s_phi,
                      const float* y, float* part, float* r, hipStream_t st) {
    if (F <= 0) return;
    CSV_REQUIRE(F <= kWMaxF && n % 64 == 0, CSV_EUNSUPPORTED, "whole-frame product shape");
    const int nk = whole_fwd_parts(n);
    whole_fwd_kernel<<<dim3(ceil_div(M, kFwdRows), nk), dim3(256),
                       (size_t)F * kFwdCols * sizeof(float), st>>>(q, x, F, n, M, part);
    CSV_HIP(hipGetLastError());
    whole_fwd_reduce_kernel<<<dim3(ceil_div(F * M, 256)), dim3(256), 0, st>>>(part, nk, F, M,
                                                                             s_phi, y, r);
    CSV_HIP(hipGetLastError());
}

void launch_whole_adj(const int8_t* q, const float* r, int F, int n, int M, float* part,
                      hipStream_t st) {
    if (F <= 0) return;
    CSV_REQUIRE(F <= kWMaxF && n % 64 == 0, CSV_EUNSUPPORTED, "whole-frame product shape");
    const int mc = whole_adj_rows(M);
    whole_adj_kernel<<<dim3(ceil_div(n, kAdjCols), ceil_div(M, mc)), dim3(256),
                       (size_t)F * mc * sizeof(float), st>>>(q, r, F, n, M, mc, part);
    CSV_HIP(hipGetLastError());
}

void launch_sum_parts(const float* part, int nparts, size_t count, float scale, float* out,
                      hipStream_t st) {
    if (!count) return;
    sum_parts_kernel<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st>>>(part, nparts,
                                                                                count, scale, out);
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
