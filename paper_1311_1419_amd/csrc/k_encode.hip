// Encoder-side kernels: measurement matrix from the counter generator, key
// frame stand-in codec, closed-loop residual measurement and quantiser.
#include "internal.h"
#include "mfma.h"
#include "philox.h"

namespace csv {

// Q[i][j] = popcount(word (i*n+j) mod 4 of philox(((i*n+j)/4, n, 0, 0), key)) - 32.
// One thread per counter (four consecutive entries of one row, n % 4 == 0).
__global__ void phi_q_kernel(int8_t* __restrict__ q, int M, int Mp, int n, uint64_t k0,
                             uint64_t k1) {
    const size_t ctr = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)Mp * n / 4;
    if (ctr >= total) return;
    const int row = (int)(ctr * 4 / n);
    char4 out = make_char4(0, 0, 0, 0);
    if (row < M) {
        uint64_t c0 = ctr, c1 = (uint64_t)n, c2 = 0, c3 = 0;
        philox4x64_10(c0, c1, c2, c3, k0, k1);
        out.x = (signed char)(__popcll(c0) - 32);
        out.y = (signed char)(__popcll(c1) - 32);
        out.z = (signed char)(__popcll(c2) - 32);
        out.w = (signed char)(__popcll(c3) - 32);
    }
    reinterpret_cast<char4*>(q)[ctr] = out;
}

void launch_phi_q(int8_t* q, int M, int Mp, int n, uint64_t k0, uint64_t k1, hipStream_t st) {
    const size_t total = (size_t)Mp * n / 4;
    phi_q_kernel<<<dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st>>>(q, M, Mp, n, k0, k1);
    CSV_HIP(hipGetLastError());
}

__global__ void fill_u64_kernel(unsigned long long* p, unsigned long long v, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

void launch_fill_u64(unsigned long long* p, unsigned long long v, int count, hipStream_t st) {
    fill_u64_kernel<<<dim3((count + 63) / 64), dim3(64), 0, st>>>(p, v, count);
    CSV_HIP(hipGetLastError());
}

// -------------------------------------------------------- key-frame codec
// Zigzag scan of an 8x8 block (JPEG order), as row*8 + col per scan index.
__constant__ int kZigzag[64] = {
    0,  1,  8,  16, 9,  2,  3,  10, 17, 24, 32, 25, 18, 11, 4,  5,
    12, 19, 26, 33, 40, 48, 41, 34, 27, 20, 13, 6,  7,  14, 21, 28,
    35, 42, 49, 56, 57, 50, 43, 36, 29, 22, 15, 23, 30, 37, 44, 51,
    58, 59, 52, 45, 38, 31, 39, 46, 53, 60, 61, 54, 47, 55, 62, 63};

// Integer DCT basis T[k][i] = round(1024 * a_k * cos(pi (2i+1) k / 16)); no
// entry is near a rounding tie, so any correctly rounded cos gives it.
__device__ inline int int_dct_entry(int k, int i) {
    const double a = k ? sqrt(2.0 / 8.0) : sqrt(1.0 / 8.0);
    return (int)rint(1024.0 * a * cos(M_PI * (2 * i + 1) * k / 16.0));
}

__device__ inline int ue_len(unsigned v) { return 2 * (31 - __clz(v + 1)) + 1; }
__device__ inline int se_len(int v) { return ue_len(2u * (unsigned)abs(v) - (v > 0 ? 1u : 0u)); }

// One wave per 8x8 block, four waves per workgroup, each wave looping over
// kKeyBlocksPerWave blocks.  Lane = pixel (r, c), then coefficient (k, l).
// Z = T X T^T is exact in 64-bit integers; level = sgn(Z) ((|Z| + 2^(s-1))
// >> s) with s = 20 + log2(step).  Bits: the nonzero mask in zigzag order
// comes from one ballot; each nonzero adds ue(run) + se(level), the block
// adds ue(nnz).  The workgroup sums its bits in LDS and adds them to the
// frame total with one atomic.
constexpr int kKeyBlocksPerWave = 4;

__global__ __launch_bounds__(256) void key_encode_kernel(const uint8_t* __restrict__ frame, int W,
                                                        int H, int qshift,
                                                        int16_t* __restrict__ levels,
                                                        unsigned long long* __restrict__ bits) {
    __shared__ int T[64];
    __shared__ int X[4][64];
    __shared__ int Y[4][64];
    __shared__ int Lv[4][64];
    __shared__ int wbits[4];
    const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
    if (tid < 64) T[tid] = int_dct_entry(tid >> 3, tid & 7);
    const int bpr = W / 8, nblk = bpr * (H / 8);
    const int r = ln >> 3, c = ln & 7;
    int acc_bits = 0;
    for (int it = 0; it < kKeyBlocksPerWave; ++it) {
        const int blk = (blockIdx.x * kKeyBlocksPerWave + it) * 4 + wv;
        const bool live = blk < nblk;
        const int by = live ? blk / bpr : 0, bx = live ? blk % bpr : 0;
        __syncthreads();   // previous round's LDS reads are done
        X[wv][ln] = live ? (int)frame[(size_t)(by * 8 + r) * W + bx * 8 + c] - 128 : 0;
        __syncthreads();
        int y = 0;   // Y[k = r][c] = sum_i T[k][i] X[i][c]
#pragma unroll
        for (int i = 0; i < 8; ++i) y += T[r * 8 + i] * X[wv][i * 8 + c];
        Y[wv][ln] = y;
        __syncthreads();
        long long z = 0;   // Z[k = r][l = c] = sum_j Y[k][j] T[l][j]
#pragma unroll
        for (int j = 0; j < 8; ++j) z += (long long)Y[wv][r * 8 + j] * T[c * 8 + j];
        const long long az = z < 0 ? -z : z;
        int lev = (int)((az + (1ll << (qshift - 1))) >> qshift);
        if (z < 0) lev = -lev;
        if (live) levels[(size_t)(by * 8 + r) * W + bx * 8 + c] = (int16_t)lev;
        Lv[wv][ln] = lev;
        __syncthreads();
        const int v = Lv[wv][kZigzag[ln]];   // lane = zigzag index
        const unsigned long long mask = __ballot(v != 0);
        int b = 0;
        if (v != 0) {
            const unsigned long long below = mask & ((1ull << ln) - 1ull);
            const int prev = below ? 63 - __clzll(below) : -1;
            b = ue_len((unsigned)(ln - prev - 1)) + se_len(v);
        }
        if (ln == 0) b += ue_len((unsigned)__popcll(mask));
        if (live) acc_bits += b;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc_bits += __shfl_down(acc_bits, off);
    if (ln == 0) wbits[wv] = acc_bits;
    __syncthreads();
    if (tid == 0 && bits)
        atomicAdd(bits, (unsigned long long)(wbits[0] + wbits[1] + wbits[2] + wbits[3]));
}

void launch_key_encode(const uint8_t* frame, int W, int H, int qshift, int16_t* levels,
                       unsigned long long* bits, hipStream_t st) {
    const int nblk = (W / 8) * (H / 8);
    key_encode_kernel<<<dim3(ceil_div(nblk, 4 * kKeyBlocksPerWave)), dim3(256), 0, st>>>(
        frame, W, H, qshift, levels, bits);
    CSV_HIP(hipGetLastError());
}

// Inverse: V = T^T (step level) T in 64-bit integers, pixel =
// clip(((V + 2^19) >> 20) + 128, 0, 255) with an arithmetic (floor) shift.
__global__ __launch_bounds__(256) void key_decode_kernel(const int16_t* __restrict__ levels, int W,
                                                        int H, int qstep,
                                                        uint8_t* __restrict__ out) {
    __shared__ int T[64];
    __shared__ long long Cq[4][64];
    __shared__ long long Wt[4][64];
    const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
    if (tid < 64) T[tid] = int_dct_entry(tid >> 3, tid & 7);
    const int bpr = W / 8, nblk = bpr * (H / 8);
    const int blk = blockIdx.x * 4 + wv;
    const bool live = blk < nblk;
    const int by = live ? blk / bpr : 0, bx = live ? blk % bpr : 0;
    const int r = ln >> 3, c = ln & 7;
    Cq[wv][ln] = live ? (long long)levels[(size_t)(by * 8 + r) * W + bx * 8 + c] * qstep : 0;
    __syncthreads();
    long long w = 0;   // Wt[k = r][j = c] = sum_l Cq[k][l] T[l][j]
#pragma unroll
    for (int l = 0; l < 8; ++l) w += Cq[wv][r * 8 + l] * T[l * 8 + c];
    Wt[wv][ln] = w;
    __syncthreads();
    long long v = 0;   // V[i = r][j = c] = sum_k T[k][i] Wt[k][j]
#pragma unroll
    for (int k = 0; k < 8; ++k) v += (long long)T[k * 8 + r] * Wt[wv][k * 8 + c];
    long long p = ((v + (1ll << 19)) >> 20) + 128;
    p = p < 0 ? 0 : (p > 255 ? 255 : p);
    if (live) out[(size_t)(by * 8 + r) * W + bx * 8 + c] = (uint8_t)p;
}

void launch_key_decode(const int16_t* levels, int W, int H, int qstep, uint8_t* out,
                       hipStream_t st) {
    const int nblk = (W / 8) * (H / 8);
    key_decode_kernel<<<dim3(ceil_div(nblk, 4)), dim3(256), 0, st>>>(levels, W, H, qstep, out);
    CSV_HIP(hipGetLastError());
}

// OCP FP8 E4M3 byte of an integer |v| <= 448: 1 sign bit, 4 exponent bits
// (bias 7), 3 mantissa bits, round to nearest, ties to even.  Integers below
// 16 are exact; above, the significand keeps its top 4 bits.
__device__ inline uint32_t int_to_e4m3(int v) {
    const uint32_t sgn = v < 0 ? 0x80u : 0u;
    const uint32_t a = (uint32_t)(v < 0 ? -v : v);
    if (a == 0u) return sgn;
    int e = 31 - __builtin_clz(a);   // a in [2^e, 2^(e+1))
    uint32_t m;                      // significand with 3 fraction bits, in [8, 16)
    if (e <= 3) {
        m = a << (3 - e);
    } else {
        const int sh = e - 3;
        m = a >> sh;
        const uint32_t rem = a & ((1u << sh) - 1u), half = 1u << (sh - 1);
        if (rem > half || (rem == half && (m & 1u))) ++m;
        if (m == 16u) {
            m = 8u;
            ++e;
        }
    }
    return sgn | ((uint32_t)(e + 7) << 3) | (m & 7u);
}

__global__ void q_e4m3_kernel(const int8_t* __restrict__ q, uint8_t* __restrict__ q8, size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) q8[i] = (uint8_t)int_to_e4m3((int)q[i]);
}

void launch_q_e4m3(const int8_t* q, uint8_t* q8, size_t count, hipStream_t st) {
    if (!count) return;
    q_e4m3_kernel<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st>>>(q, q8, count);
    CSV_HIP(hipGetLastError());
}

// ------------------------------------------------------------ measurement
// y~ = Q r for a tile of 32 blocks, in one of three forms:
//   FORM 0 (exact): the residual (frame - decoded key, zero outside the
//          frame) is staged in LDS as bf16 and Q (int8) is widened to bf16
//          in registers; both are exact (|r| <= 255, |Q| <= 32) and so is
//          the FP32 accumulation (every partial sum < 2^24 for n <= 2048);
//   FORM 1 (int8): two byte planes, the digits h = r >> 4 (in [-16, 15]) and
//          l = r & 15 (in [0, 15]) of r = 16 h + l; Q times each plane on
//          int8 MFMA with int32 accumulation, y~ = 16 Q h + Q l = Q r;
//   FORM 2 (fp8): one plane of E4M3 residuals times the E4M3 copy of Q on
//          FP8 MFMA; every operand is an integer and every partial sum is
//          below 2^24, so the FP32 accumulator holds the exact integer sum
//          of e4m3(Q) e4m3(r).
// Staging moves 8 pixels per load (W % 8 == 0 keeps a group inside or
// outside the frame and aligned) with the loads of four groups in flight.
// Each wave computes 32-row M tiles with 32x32x16 MFMA; operand layout of
// the 32x32x16 MFMA: lane l, elements e = 0..7 carry row (A) or column (B)
// l % 32 and K index 8 (l / 32) + e.
template <int B, int FORM>
struct MeasureLayout {
    static constexpr int n = B * B;
    static constexpr int EB = FORM == 0 ? 2 : 1;                  // staged bytes per residual
    static constexpr int LD = FORM == 0 ? 2 * n + 16 : n + 8;     // bytes per block; pads spread banks
    static constexpr int PLANES = FORM == 1 ? 2 : 1;
    static constexpr size_t PLANE = (size_t)32 * LD;
    static constexpr size_t LDS = PLANE * PLANES;
};

__device__ inline int byte_of(uint2 w, int i) {
    return (int)(((i < 4 ? w.x : w.y) >> (8 * (i & 3))) & 0xffu);
}

template <int B, int FORM>
__global__ __launch_bounds__(256) void measure_kernel(const int8_t* __restrict__ q,
                                                      const uint8_t* __restrict__ q8, int Mp,
                                                      const uint8_t* __restrict__ frames,
                                                      int n_frames, size_t frame_stride,
                                                      const uint8_t* __restrict__ key, int W, int H,
                                                      int nbx, int nb, int32_t* __restrict__ y) {
    using L = MeasureLayout<B, FORM>;
    constexpr int n = L::n;
    extern __shared__ __attribute__((aligned(16))) uint8_t res[];   // [PLANES][32][LD]
    const int tid = threadIdx.x;
    const int total = n_frames * nb;
    const int gb0 = blockIdx.x * 32;
    constexpr int PER = 32 * n / 8 / 256;   // 8-pixel groups per thread: 16 (B=32) or 4 (B=16)
    constexpr int U = 4;
    static_assert(PER % U == 0, "staging rounds");
#pragma unroll 1
    for (int base = 0; base < PER; base += U) {
        uint2 fv[U], kv[U];
        size_t dst[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int item = tid + 256 * (base + u);
            const int j = item / (n / 8);
            const int rem = item - j * (n / 8);
            const int r = rem / (B / 8), c8 = (rem - r * (B / 8)) * 8;
            const int gb = gb0 + j;
            fv[u] = make_uint2(0u, 0u);
            kv[u] = make_uint2(0u, 0u);
            if (gb < total) {
                const int t = gb / nb, b = gb - t * nb;
                const int py = (b / nbx) * B + r, px = (b % nbx) * B + c8;
                if (py < H && px < W) {
                    fv[u] = *reinterpret_cast<const uint2*>(frames + t * frame_stride + (size_t)py * W + px);
                    kv[u] = *reinterpret_cast<const uint2*>(key + (size_t)py * W + px);
                }
            }
            dst[u] = (size_t)j * L::LD + (size_t)(r * B + c8) * L::EB;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = byte_of(fv[u], i) - byte_of(kv[u], i);
            if constexpr (FORM == 0) {
                u16x8 o;
#pragma unroll
                for (int i = 0; i < 8; ++i) o[i] = int_to_bf16_exact(v[i]);
                *reinterpret_cast<u16x8*>(res + dst[u]) = o;
            } else if constexpr (FORM == 1) {
                uint2 wh = make_uint2(0u, 0u), wl = make_uint2(0u, 0u);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    wh.x |= ((uint32_t)(v[i] >> 4) & 0xffu) << (8 * i);
                    wh.y |= ((uint32_t)(v[4 + i] >> 4) & 0xffu) << (8 * i);
                    wl.x |= ((uint32_t)(v[i] & 15)) << (8 * i);
                    wl.y |= ((uint32_t)(v[4 + i] & 15)) << (8 * i);
                }
                *reinterpret_cast<uint2*>(res + dst[u]) = wh;
                *reinterpret_cast<uint2*>(res + L::PLANE + dst[u]) = wl;
            } else {
                uint2 w8 = make_uint2(0u, 0u);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    w8.x |= int_to_e4m3(v[i]) << (8 * i);
                    w8.y |= int_to_e4m3(v[4 + i]) << (8 * i);
                }
                *reinterpret_cast<uint2*>(res + dst[u]) = w8;
            }
        }
    }
    __syncthreads();
    const int wv = tid >> 6, ln = tid & 63, col = ln & 31, half = ln >> 5;
    for (int mt = wv; mt < Mp / 32; mt += 4) {
        const size_t qoff = (size_t)(mt * 32 + col) * n + 8 * half;
        const uint8_t* rrow = res + (size_t)col * L::LD + (size_t)8 * half * L::EB;
        int32_t out[16];
        if constexpr (FORM == 0) {
            floatx16 acc = {};
#pragma unroll 8
            for (int s = 0; s < n / 16; ++s) {
                const bf16x8 a = int8x8_to_bf16x8(*reinterpret_cast<const uint2*>(q + qoff + 16 * s));
                const bf16x8 b = *reinterpret_cast<const bf16x8*>(rrow + 16 * s * L::EB);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) out[r] = (int32_t)acc[r];
        } else if constexpr (FORM == 1) {
            intx16 ah = {}, al = {};
#pragma unroll 8
            for (int s = 0; s < n / 16; ++s) {
                const long a = *reinterpret_cast<const long*>(q + qoff + 16 * s);
                const long bh = *reinterpret_cast<const long*>(rrow + 16 * s);
                const long bl = *reinterpret_cast<const long*>(rrow + L::PLANE + 16 * s);
                ah = __builtin_amdgcn_mfma_i32_32x32x16_i8(a, bh, ah, 0, 0, 0);
                al = __builtin_amdgcn_mfma_i32_32x32x16_i8(a, bl, al, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) out[r] = 16 * ah[r] + al[r];
        } else {
            floatx16 acc = {};
#pragma unroll 8
            for (int s = 0; s < n / 16; ++s) {
                const long a = *reinterpret_cast<const long*>(q8 + qoff + 16 * s);
                const long b = *reinterpret_cast<const long*>(rrow + 16 * s);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) out[r] = (int32_t)acc[r];
        }
        const int gb = gb0 + col;
        if (gb < total) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = mt * 32 + 8 * (r / 4) + 4 * half + (r % 4);
                y[(size_t)gb * Mp + m] = out[r];
            }
        }
    }
}

template <int B, int FORM>
static void launch_measure_form(const Shape& s, const int8_t* q, const uint8_t* q8,
                                const uint8_t* frames, int n_frames, size_t frame_stride,
                                const uint8_t* key, int32_t* y, hipStream_t st) {
    const int total = n_frames * s.nb;
    const size_t lds = MeasureLayout<B, FORM>::LDS;
    auto* fn = &measure_kernel<B, FORM>;
    ensure_lds_limit<&measure_kernel<B, FORM>>(lds);
    fn<<<dim3(ceil_div(total, 32)), dim3(256), lds, st>>>(q, q8, s.Mp, frames, n_frames,
                                                           frame_stride, key, s.W, s.H, s.nbx,
                                                           s.nb, y);
    CSV_HIP(hipGetLastError());
}

template <int B>
static void launch_measure_b(const Shape& s, const int8_t* q, const uint8_t* q8,
                             const uint8_t* frames, int n_frames, size_t frame_stride,
                             const uint8_t* key, int32_t* y, hipStream_t st) {
    if (s.flags & CSV_FLAG_MEASURE_INT8)
        launch_measure_form<B, 1>(s, q, q8, frames, n_frames, frame_stride, key, y, st);
    else if (s.flags & CSV_FLAG_MEASURE_FP8)
        launch_measure_form<B, 2>(s, q, q8, frames, n_frames, frame_stride, key, y, st);
    else
        launch_measure_form<B, 0>(s, q, q8, frames, n_frames, frame_stride, key, y, st);
}

void launch_measure(const Shape& s, const int8_t* q, const uint8_t* q8, const uint8_t* frames,
                    int n_frames, size_t frame_stride, const uint8_t* key, int32_t* y_scratch,
                    hipStream_t st) {
    // y_scratch: (n_frames * nb) x Mp int32
    const int total = n_frames * s.nb;
    if (total == 0) return;
    CSV_REQUIRE((reinterpret_cast<uintptr_t>(frames) | reinterpret_cast<uintptr_t>(key)) % 8 == 0,
                CSV_EINVAL, "frame buffers must be 8-byte aligned");
    if (s.B == 16)
        launch_measure_b<16>(s, q, q8, frames, n_frames, frame_stride, key, y_scratch, st);
    else
        launch_measure_b<32>(s, q, q8, frames, n_frames, frame_stride, key, y_scratch, st);
}

// Block-floating-point 8-bit quantiser, one wave per block: m = max|y~|,
// e = min{e >= 0 : (m + h(e)) >> e <= 127} with h(0) = 0, h(e) = 2^(e-1);
// code = sgn(y~) ((|y~| + h(e)) >> e).  raw (the no-quantiser test form):
// y~ itself is stored as int32 at `codes` and the exponent is 0.
__global__ __launch_bounds__(256) void quantise_kernel(const int32_t* __restrict__ y, int M, int Mp,
                                                      int total, int8_t* __restrict__ codes,
                                                      uint8_t* __restrict__ exps,
                                                      int32_t* __restrict__ y_out, int raw) {
    const int gb = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int ln = threadIdx.x & 63;
    if (gb >= total) return;   // whole wave leaves together
    const int32_t* row = y + (size_t)gb * Mp;
    if (raw) {
        int32_t* c32 = reinterpret_cast<int32_t*>(codes);
        for (int m = ln; m < M; m += 64) {
            c32[(size_t)gb * M + m] = row[m];
            if (y_out) y_out[(size_t)gb * M + m] = row[m];
        }
        if (ln == 0) exps[gb] = 0;
        return;
    }
    int mx = 0;
    for (int m = ln; m < M; m += 64) mx = max(mx, abs(row[m]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off));
    int e = 0;
    while (((mx + (e ? (1 << (e - 1)) : 0)) >> e) > 127) ++e;
    const int h = e ? (1 << (e - 1)) : 0;
    for (int m = ln; m < M; m += 64) {
        const int v = row[m];
        const int a = (abs(v) + h) >> e;
        codes[(size_t)gb * M + m] = (int8_t)(v < 0 ? -a : a);
        if (y_out) y_out[(size_t)gb * M + m] = v;
    }
    if (ln == 0) exps[gb] = (uint8_t)e;
}

void launch_quantise(const int32_t* y, int M, int Mp, int total, int8_t* codes, uint8_t* exps,
                     int32_t* y_out, hipStream_t st, bool raw) {
    if (total == 0) return;
    CSV_REQUIRE(!raw || reinterpret_cast<uintptr_t>(codes) % 4 == 0, CSV_EINVAL,
                "unquantised measurements need a 4-byte aligned codes buffer");
    quantise_kernel<<<dim3(ceil_div(total, 4)), dim3(256), 0, st>>>(y, M, Mp, total, codes, exps,
                                                                    y_out, raw ? 1 : 0);
    CSV_HIP(hipGetLastError());
}

}  // namespace csv
