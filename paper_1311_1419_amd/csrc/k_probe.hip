// Achievable device ceilings (csv_probe_ceilings): short microbenchmarks
// that a roofline fraction is read against besides the datasheet peaks.
//   MFMA:  four independent 32x32x16 BF16 chains per wave, 8 waves per CU;
//   L2:    every CU streams the same 1 MiB buffer (it stays in each XCD's
//          L2), 16-byte loads, eight in flight per lane;
//   HBM:   the CUs stream disjoint parts of a 1 GiB buffer once;
//   LDS:   ds_read_b128 over 64 KiB per CU.
// Every index stays inside its buffer by construction (see each kernel).
#include <algorithm>

#include "internal.h"
#include "mfma.h"

namespace csv {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 gu32x4;

constexpr int kProbeThreads = 512;

// n16: buffer length in 16-byte words, a multiple of kProbeThreads * 8.
// Index base + u * 512 + tid + rot < 2 n16 and is folded once, so < n16.
__global__ __launch_bounds__(kProbeThreads) void probe_l2_kernel(const u32x4* __restrict__ buf,
                                                                 size_t n16, int reps,
                                                                 u32x4* __restrict__ sink) {
    const gu32x4* g = (const gu32x4*)buf;
    u32x4 acc = {0, 0, 0, 0};
    const int tid = threadIdx.x;
    const size_t rot = ((size_t)blockIdx.x * 4096) % n16;
    for (int r = 0; r < reps; ++r) {
        for (size_t base = 0; base < n16; base += (size_t)kProbeThreads * 8) {
            u32x4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                size_t i = base + (size_t)u * kProbeThreads + tid + rot;
                if (i >= n16) i -= n16;
                v[u] = g[i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc ^= v[u];
        }
    }
    sink[(size_t)blockIdx.x * kProbeThreads + tid] = acc;
}

// Grid-stride read of n16 words, eight loads in flight per lane.
__global__ __launch_bounds__(kProbeThreads) void probe_hbm_kernel(const u32x4* __restrict__ buf,
                                                                  size_t n16,
                                                                  u32x4* __restrict__ sink) {
    const gu32x4* g = (const gu32x4*)buf;
    u32x4 acc = {0, 0, 0, 0};
    const size_t stride = (size_t)gridDim.x * kProbeThreads;
    size_t i = (size_t)blockIdx.x * kProbeThreads + threadIdx.x;
    for (; i + 7 * stride < n16; i += 8 * stride) {
        u32x4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = g[i + u * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc ^= v[u];
    }
    for (; i < n16; i += stride) acc ^= g[i];
    sink[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = acc;
}

// 64 KiB of LDS; row (k + w) & 63 of 64 rows of 64 words.
__global__ __launch_bounds__(kProbeThreads) void probe_lds_kernel(int reps,
                                                                  u32x4* __restrict__ sink) {
    __shared__ u32x4 s[64 * 64];
    const int tid = threadIdx.x;
    for (int i = tid; i < 64 * 64; i += kProbeThreads)
        s[i] = u32x4{(unsigned)i, (unsigned)i * 3u, (unsigned)i * 5u, (unsigned)i * 7u};
    __syncthreads();
    u32x4 acc = {0, 0, 0, 0};
    const int w = tid >> 6, ln = tid & 63;
    for (int r = 0; r < reps; ++r) {
#pragma unroll 8
        for (int k = 0; k < 64; ++k) acc ^= s[((k + w) & 63) * 64 + ln];
    }
    sink[(size_t)blockIdx.x * kProbeThreads + tid] = acc;
}

__global__ __launch_bounds__(kProbeThreads) void probe_mfma_kernel(int reps,
                                                                   float* __restrict__ sink) {
    const int tid = threadIdx.x;
    u16x8 a;
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = (uint16_t)(0x3f80 + ((tid + e) & 1));   // 1.0 or 1.0078
    const bf16x8 ab = __builtin_bit_cast(bf16x8, a);
    floatx16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int r = 0; r < reps; ++r) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, ab, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, ab, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, ab, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, ab, c3, 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += c0[i] + c1[i] + c2[i] + c3[i];
    sink[(size_t)blockIdx.x * kProbeThreads + tid] = s;
}

namespace {
struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() {
        CSV_HIP(hipEventCreate(&a));
        CSV_HIP(hipEventCreate(&b));
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    // best of `reps` timed runs of f (milliseconds)
    template <class F>
    double best(int reps, F&& f, hipStream_t st) {
        f();   // warm-up
        double ms = 1e30;
        for (int r = 0; r < reps; ++r) {
            CSV_HIP(hipEventRecord(a, st));
            f();
            CSV_HIP(hipEventRecord(b, st));
            CSV_HIP(hipEventSynchronize(b));
            float t = 0.f;
            CSV_HIP(hipEventElapsedTime(&t, a, b));
            ms = std::min(ms, (double)t);
        }
        return ms;
    }
};
}  // namespace

void probe_ceilings(Ctx* c, int cus, csv_ceilings* out) {
    hipStream_t st = nullptr;
    const size_t sink_words = (size_t)cus * 4 * kProbeThreads;
    const size_t l2_bytes = (size_t)1 << 20, hbm_bytes = (size_t)1 << 30;
    void* sink = ctx_alloc(c, sink_words * 16);
    void* l2buf = nullptr;
    void* hbm = nullptr;
    try {
        l2buf = ctx_alloc(c, l2_bytes);
        hbm = ctx_alloc(c, hbm_bytes);
        CSV_HIP(hipMemsetAsync(l2buf, 1, l2_bytes, st));
        CSV_HIP(hipMemsetAsync(hbm, 3, hbm_bytes, st));
        Timer t;
        u32x4* sk = static_cast<u32x4*>(sink);
        {   // MFMA: cus workgroups x 8 waves x 4 chains
            const int reps = 20000;
            const double ms = t.best(3, [&] {
                probe_mfma_kernel<<<dim3(cus), dim3(kProbeThreads), 0, st>>>(reps,
                                                                           static_cast<float*>(sink));
                CSV_HIP(hipGetLastError());
            }, st);
            out->mfma_bf16_tflops = (double)cus * 8 * reps * 4 * 32768.0 / (ms * 1e-3) / 1e12;
        }
        {   // L2: cus workgroups each stream the same 1 MiB
            const size_t n16 = l2_bytes / 16;
            const int reps = 40;
            const double ms = t.best(3, [&] {
                probe_l2_kernel<<<dim3(cus), dim3(kProbeThreads), 0, st>>>(
                    static_cast<const u32x4*>(l2buf), n16, reps, sk);
                CSV_HIP(hipGetLastError());
            }, st);
            out->l2_read_tbs = (double)cus * reps * l2_bytes / (ms * 1e-3) / 1e12;
        }
        {   // HBM: 1 GiB read once by 4 workgroups per CU
            const size_t n16 = hbm_bytes / 16;
            const double ms = t.best(3, [&] {
                probe_hbm_kernel<<<dim3(cus * 4), dim3(kProbeThreads), 0, st>>>(
                    static_cast<const u32x4*>(hbm), n16, sk);
                CSV_HIP(hipGetLastError());
            }, st);
            out->hbm_read_tbs = (double)hbm_bytes / (ms * 1e-3) / 1e12;
        }
        {   // LDS
            const int reps = 2000;
            const double ms = t.best(3, [&] {
                probe_lds_kernel<<<dim3(cus), dim3(kProbeThreads), 0, st>>>(reps, sk);
                CSV_HIP(hipGetLastError());
            }, st);
            out->lds_read_tbs = (double)cus * kProbeThreads * reps * 64 * 16 / (ms * 1e-3) / 1e12;
        }
        out->compute_units = cus;
    } catch (...) {
        (void)hipDeviceSynchronize();
        ctx_free(c, hbm, hbm_bytes);
        ctx_free(c, l2buf, l2_bytes);
        ctx_free(c, sink, sink_words * 16);
        throw;
    }
    CSV_HIP(hipDeviceSynchronize());
    ctx_free(c, hbm, hbm_bytes);
    ctx_free(c, l2buf, l2_bytes);
    ctx_free(c, sink, sink_words * 16);
}

}  // namespace csv
