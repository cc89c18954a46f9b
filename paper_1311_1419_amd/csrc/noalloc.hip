// csv_measure_frame_noalloc: the measurement of one CS frame (the residual
// against the decoded key frame, eqs. (2)-(3); y~ = Q r per block; the 8-bit
// quantiser) without any device allocation, for callers that cannot
// allocate.  Its working memory is one file-scope device array per GPU:
//   [padded Q: Mp x n int8][Q as E4M3 (FP8 form only): Mp x n][y~: N_b x Mp int32]
// Host code never passes the array's name to a kernel: its device address
// is looked up once per device with hipGetSymbolAddress and kept.
#include <array>
#include <mutex>

#include "internal.h"

// per device, held until the process ends (file scope, outside the
// namespace whose scratch() manages context buffers)
constexpr size_t kNoAllocBytes = (size_t)16 << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace csv {

namespace {

std::mutex g_mu;
std::array<void*, 64> g_ptr{};   // scratch's address on each device ordinal

void* scratch_address(int dev) {
    CSV_REQUIRE(dev >= 0 && dev < (int)g_ptr.size(), CSV_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        CSV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(::scratch)));
        CSV_REQUIRE(p != nullptr, CSV_EHIP, "scratch symbol has no device address");
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

// Rows m < M of Q (M x n, the caller's) into the Mp x n copy, rows M..Mp-1
// zero: the layout the measurement kernel reads.
__global__ void pad_q_kernel(const int8_t* __restrict__ q, int M, int Mp, int n,
                             int8_t* __restrict__ qp) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)Mp * n) return;
    qp[i] = i < (size_t)M * n ? q[i] : (int8_t)0;
}

size_t al256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

// Set-up of the allocation-free entry point on `dev` (the current device):
// the first lookup of the array's address loads its code object there.
void noalloc_setup(int dev) { (void)scratch_address(dev); }

size_t noalloc_scratch_need(const Shape& s) {
    const size_t qb = al256((size_t)s.Mp * s.n);
    return qb + ((s.flags & CSV_FLAG_MEASURE_FP8) ? qb : 0) + (size_t)s.nb * s.Mp * 4;
}

}  // namespace csv

using namespace csv;

extern "C" int csv_measure_frame_noalloc(const csv_params* p, const int8_t* q,
                                         const uint8_t* frame, const uint8_t* key_decoded,
                                         int32_t* y_out, int8_t* codes, uint8_t* exps,
                                         void* stream) {
    try {
        CSV_REQUIRE(q && frame && key_decoded && codes && exps, CSV_EINVAL, "NULL argument");
        const Shape s = resolve(p);
        CSV_REQUIRE(!(s.flags & CSV_FLAG_WHOLE_FRAME), CSV_EUNSUPPORTED,
                    "whole-frame measurement has no allocation-free form");
        const size_t need = noalloc_scratch_need(s);
        CSV_REQUIRE(need <= kNoAllocBytes, CSV_EINVAL,
                    "frame needs " + std::to_string(need) +
                        " bytes of measurement scratch, above the allocation-free limit of " +
                        std::to_string(kNoAllocBytes) + " (use csv_measure_frame)");
        int dev = 0;
        CSV_HIP(hipGetDevice(&dev));
        uint8_t* base = static_cast<uint8_t*>(scratch_address(dev));
        hipStream_t st = static_cast<hipStream_t>(stream);
        const size_t qb = al256((size_t)s.Mp * s.n);
        int8_t* qp = reinterpret_cast<int8_t*>(base);
        uint8_t* q8 = nullptr;
        size_t off = qb;
        if (s.flags & CSV_FLAG_MEASURE_FP8) {
            q8 = base + off;
            off += qb;
        }
        int32_t* y = reinterpret_cast<int32_t*>(base + off);
        const size_t qn = (size_t)s.Mp * s.n;
        pad_q_kernel<<<dim3((unsigned)((qn + 255) / 256)), dim3(256), 0, st>>>(q, s.M, s.Mp, s.n,
                                                                              qp);
        CSV_HIP(hipGetLastError());
        if (q8) launch_q_e4m3(qp, q8, qn, st);
        launch_measure(s, qp, q8, frame, 1, (size_t)s.W * s.H, key_decoded, y, st);
        launch_quantise(y, s.M, s.Mp, s.nb, codes, exps, y_out, st,
                        (s.flags & CSV_FLAG_NO_QUANT) != 0);
        return CSV_OK;
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    } catch (const std::exception& e) {
        return fail(CSV_EINVAL, e.what());
    }
}
