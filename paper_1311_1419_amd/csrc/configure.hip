// Parameter configurator (include/csv_config.h): for every candidate GOP
// size G and measurement count M, the coder runs over a calibration clip
// (encode and decode of all its GOPs as one batch each), and the total
// compression ratio (Table I) and the decoded PSNR are measured; the
// candidate of largest total CR that meets the PSNR floor is chosen
// (Sections 2-3, Fig. 6).
#include <cmath>
#include <cstring>
#include <functional>

#include "csv_config.h"
#include "internal.h"

namespace csv {

// Per-frame sum of squared differences: grid (chunks, frames), 256 threads,
// 8 pixels per load (frame_px % 8 == 0), one 64-bit atomic per workgroup.
__global__ __launch_bounds__(256) void sse_kernel(const uint8_t* __restrict__ a,
                                                  const uint8_t* __restrict__ b, size_t frame_px,
                                                  unsigned long long* __restrict__ sse) {
    __shared__ unsigned long long part[4];
    const size_t f = blockIdx.y;
    const uint8_t* pa = a + f * frame_px;
    const uint8_t* pb = b + f * frame_px;
    unsigned long long acc = 0;
    for (size_t i = ((size_t)blockIdx.x * 256 + threadIdx.x) * 8; i < frame_px;
         i += (size_t)gridDim.x * 256 * 8) {
        const uint2 x = *reinterpret_cast<const uint2*>(pa + i);
        const uint2 y = *reinterpret_cast<const uint2*>(pb + i);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int d0 = (int)((x.x >> (8 * k)) & 0xffu) - (int)((y.x >> (8 * k)) & 0xffu);
            const int d1 = (int)((x.y >> (8 * k)) & 0xffu) - (int)((y.y >> (8 * k)) & 0xffu);
            acc += (unsigned long long)(d0 * d0) + (unsigned long long)(d1 * d1);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) part[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&sse[f], part[0] + part[1] + part[2] + part[3]);
}

static void launch_sse(const uint8_t* a, const uint8_t* b, int n_frames, int W, int H,
                       unsigned long long* sse, hipStream_t st) {
    if (n_frames <= 0) return;
    CSV_REQUIRE(W % 8 == 0 && ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) % 8) == 0,
                CSV_EINVAL, "frames must be 8-byte aligned with W a multiple of 8");
    const size_t px = (size_t)W * H;
    launch_fill_u64(sse, 0ull, n_frames, st);
    const unsigned chunks = (unsigned)std::min<size_t>((px / 8 + 255) / 256, 64);
    sse_kernel<<<dim3(chunks, (unsigned)n_frames), dim3(256), 0, st>>>(a, b, px, sse);
    CSV_HIP(hipGetLastError());
}

static double psnr_of(unsigned long long sse, size_t px) {
    return sse == 0 ? 99.99 : 10.0 * std::log10(255.0 * 255.0 * (double)px / (double)sse);
}

static void configure(Ctx* c, const csv_params& base, const uint8_t* clip, int F,
                      const int32_t* gops, int n_g, const int32_t* ms, int n_m, double floor_db,
                      csv_config_point* points, int32_t* best, hipStream_t st) {
    const size_t hw = (size_t)base.width * base.height;
    int chosen = -1;
    for (int gi = 0; gi < n_g; ++gi) {
        for (int mi = 0; mi < n_m; ++mi) {
            const int G = gops[gi], M = ms[mi];
            CSV_REQUIRE(G >= 1, CSV_EINVAL, "GOP sizes must be at least 1");
            // the clip's GOPs: consecutive runs of G frames, the last shorter
            std::vector<Shape> shapes;
            std::vector<int> start;
            for (int f0 = 0; f0 < F; f0 += G) {
                csv_params p = base;
                p.gop = std::min(G, F - f0);
                p.m = M;
                shapes.push_back(resolve(&p));
                start.push_back(f0);
            }
            const int count = (int)shapes.size();
            // coded streams and decoded clip in one scratch buffer
            auto al = [](size_t v) { return (v + 255) / 256 * 256; };
            size_t bytes = al(hw * F) + al((size_t)F * 8);
            for (const Shape& s : shapes)
                bytes += al(hw * 2) + al((size_t)(s.G - 1) * s.nb * s.M) +
                         al((size_t)(s.G - 1) * s.nb) + al(16);
            char* buf = static_cast<char*>(scratch(c, "cfg", bytes));
            size_t off = 0;
            auto take = [&](size_t v) {
                char* p = buf + off;
                off += al(v);
                return p;
            };
            uint8_t* dec = reinterpret_cast<uint8_t*>(take(hw * F));
            unsigned long long* sse = reinterpret_cast<unsigned long long*>(take((size_t)F * 8));
            std::vector<csv_gop_stream> gs(count);
            std::vector<const uint8_t*> in(count);
            std::vector<uint8_t*> out(count);
            for (int k = 0; k < count; ++k) {
                const Shape& s = shapes[k];
                gs[k].key_levels = reinterpret_cast<int16_t*>(take(hw * 2));
                gs[k].codes = reinterpret_cast<int8_t*>(take((size_t)(s.G - 1) * s.nb * s.M));
                gs[k].exps = reinterpret_cast<uint8_t*>(take((size_t)(s.G - 1) * s.nb));
                gs[k].bits = reinterpret_cast<uint64_t*>(take(16));
                in[k] = clip + (size_t)start[k] * hw;
                out[k] = dec + (size_t)start[k] * hw;
            }
            encode_gops(c, count, shapes.data(), in.data(), gs.data(), st);
            decode_gops(c, count, shapes.data(), gs.data(), out.data(), nullptr, nullptr, st);
            launch_sse(clip, dec, F, base.width, base.height, sse, st);
            std::vector<unsigned long long> sse_h(F);
            std::vector<uint64_t> bits_h(2 * (size_t)count);
            CSV_HIP(hipMemcpyAsync(sse_h.data(), sse, (size_t)F * 8, hipMemcpyDeviceToHost, st));
            for (int k = 0; k < count; ++k)
                CSV_HIP(hipMemcpyAsync(&bits_h[2 * k], gs[k].bits, 16, hipMemcpyDeviceToHost, st));
            CSV_HIP(hipStreamSynchronize(st));
            csv_config_point& pt = points[gi * n_m + mi];
            std::memset(&pt, 0, sizeof(pt));
            pt.gop = G;
            pt.m = shapes[0].M;
            int n_cs = 0;
            double ps_all = 0.0, ps_cs = 0.0;
            for (int k = 0; k < count; ++k) {
                pt.bits_key += bits_h[2 * k];
                pt.bits_cs += bits_h[2 * k + 1];
                for (int t = 0; t < shapes[k].G; ++t) {
                    const double ps = psnr_of(sse_h[start[k] + t], hw);
                    ps_all += ps;
                    if (t > 0) {
                        ps_cs += ps;
                        ++n_cs;
                    }
                }
            }
            const double raw_key = 8.0 * hw * count, raw_cs = 8.0 * hw * (F - count);
            pt.cr_total = (raw_key + raw_cs) / (double)(pt.bits_key + pt.bits_cs);
            pt.cr_key = raw_key / (double)pt.bits_key;
            pt.cr_cs = pt.bits_cs ? raw_cs / (double)pt.bits_cs : 0.0;
            pt.psnr_all = ps_all / F;
            pt.psnr_cs = n_cs ? ps_cs / n_cs : 0.0;
            pt.meets_floor = pt.psnr_all >= floor_db ? 1 : 0;
            const int idx = gi * n_m + mi;
            if (pt.meets_floor && (chosen < 0 || pt.cr_total > points[chosen].cr_total)) chosen = idx;
        }
    }
    *best = chosen;
}

}  // namespace csv

using namespace csv;

static int guarded_c(const std::function<void()>& f) {
    try {
        f();
        return CSV_OK;
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(CSV_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(CSV_EINVAL, e.what());
    }
}

extern "C" {

int csv_configure(csv_ctx* ctx, const csv_params* base, const uint8_t* clip, int32_t n_frames,
                  const int32_t* gops, int32_t n_g, const int32_t* ms, int32_t n_m,
                  double psnr_floor, csv_config_point* points, int32_t* best, void* stream) {
    return guarded_c([&] {
        CSV_REQUIRE(ctx && base && clip && gops && ms && points && best, CSV_EINVAL, "NULL argument");
        CSV_REQUIRE(n_frames >= 1 && n_g >= 1 && n_m >= 1, CSV_EINVAL,
                    "need at least one frame and one candidate");
        CSV_REQUIRE(!(base->flags & CSV_FLAG_NO_QUANT), CSV_EUNSUPPORTED,
                    "the configurator counts quantised bits: CSV_FLAG_NO_QUANT is a decoder test "
                    "hook");
        std::lock_guard<std::mutex> lk(ctx->mu);
        CSV_HIP(hipSetDevice(ctx->impl.device));
        configure(&ctx->impl, *base, clip, n_frames, gops, n_g, ms, n_m, psnr_floor, points, best,
                  static_cast<hipStream_t>(stream));
    });
}

int csv_frame_sse(csv_ctx* ctx, const uint8_t* a, const uint8_t* b, int32_t n_frames,
                  int32_t width, int32_t height, uint64_t* sse, void* stream) {
    return guarded_c([&] {
        CSV_REQUIRE(ctx && a && b && sse, CSV_EINVAL, "NULL argument");
        CSV_REQUIRE(n_frames >= 0 && width > 0 && height > 0, CSV_EINVAL, "bad sizes");
        std::lock_guard<std::mutex> lk(ctx->mu);
        CSV_HIP(hipSetDevice(ctx->impl.device));
        launch_sse(a, b, n_frames, width, height, reinterpret_cast<unsigned long long*>(sse),
                   static_cast<hipStream_t>(stream));
    });
}

}  // extern "C"
