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

}  // namespace csv
