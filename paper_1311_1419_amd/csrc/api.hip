// Host side of the C ABI: validation, context and per-stream operator
// caches, scratch management and the encode / decode orchestration.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include <map>
#include <tuple>

#include "internal.h"

namespace csv {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

template <class F>
static int guarded(F&& f) {
    try {
        f();
        return CSV_OK;
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(CSV_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(CSV_EINVAL, e.what());
    } catch (...) {
        return fail(CSV_EINVAL, "unknown error");
    }
}

// ------------------------------------------------------------ parameters
static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

Shape resolve(const csv_params* p) {
    CSV_REQUIRE(p != nullptr, CSV_EINVAL, "params is NULL");
    Shape s{};
    CSV_REQUIRE(p->width > 0 && p->height > 0, CSV_EINVAL, "frame size must be positive");
    CSV_REQUIRE(p->width % 8 == 0 && p->height % 8 == 0, CSV_EINVAL,
                "frame width and height must be multiples of 8");
    CSV_REQUIRE(p->width <= 16384 && p->height <= 16384, CSV_EINVAL, "frame too large");
    CSV_REQUIRE(p->block == 16 || p->block == 32, CSV_EINVAL, "block must be 16 or 32");
    CSV_REQUIRE(p->gop >= 1 && p->gop <= 1024, CSV_EINVAL, "gop must be in [1, 1024]");
    CSV_REQUIRE(is_pow2(p->key_qstep) && p->key_qstep <= 256, CSV_EINVAL,
                "key_qstep must be a power of two in [1, 256]");
    CSV_REQUIRE(p->iters >= 1 && p->iters <= 100000, CSV_EINVAL, "iters must be in [1, 100000]");
    CSV_REQUIRE(p->lambda_frac >= 0.f && std::isfinite(p->lambda_frac), CSV_EINVAL,
                "lambda_frac must be finite and >= 0");
    CSV_REQUIRE(p->precision == CSV_FP32 || p->precision == CSV_BF16, CSV_EINVAL,
                "precision must be CSV_FP32 or CSV_BF16");
    CSV_REQUIRE((p->flags & ~(CSV_FLAG_ISTA | CSV_FLAG_LAMBDA_PIXEL_DOMAIN |
                              CSV_FLAG_MEASURE_INT8 | CSV_FLAG_MEASURE_FP8 | CSV_FLAG_TV |
                              CSV_FLAG_WHOLE_FRAME | CSV_FLAG_MONOTONE | CSV_FLAG_NO_QUANT)) == 0,
                CSV_EINVAL, "unknown flag bits");
    CSV_REQUIRE(!(p->flags & CSV_FLAG_MONOTONE) || !(p->flags & (CSV_FLAG_ISTA | CSV_FLAG_TV)),
                CSV_EINVAL, "CSV_FLAG_MONOTONE selects the l1 solver: not with ISTA or TV");
    CSV_REQUIRE(!(p->flags & CSV_FLAG_NO_QUANT) ||
                    !(p->flags & (CSV_FLAG_TV | CSV_FLAG_WHOLE_FRAME)),
                CSV_EUNSUPPORTED, "CSV_FLAG_NO_QUANT covers block DCT-l1 recovery only");
    CSV_REQUIRE(!(p->flags & CSV_FLAG_WHOLE_FRAME) ||
                    !(p->flags & (CSV_FLAG_MEASURE_INT8 | CSV_FLAG_MEASURE_FP8)),
                CSV_EINVAL, "whole-frame measurement is exact integer only");
    CSV_REQUIRE(!(p->flags & CSV_FLAG_WHOLE_FRAME) || p->gop <= 32, CSV_EUNSUPPORTED,
                "whole-frame measurement supports GOPs of at most 32 frames");
    CSV_REQUIRE((p->flags & (CSV_FLAG_MEASURE_INT8 | CSV_FLAG_MEASURE_FP8)) !=
                    (CSV_FLAG_MEASURE_INT8 | CSV_FLAG_MEASURE_FP8),
                CSV_EINVAL, "at most one measurement form flag");
    s.W = p->width;
    s.H = p->height;
    s.G = p->gop;
    s.B = p->block;
    const bool whole = (p->flags & CSV_FLAG_WHOLE_FRAME) != 0;
    // whole frame: one vector of W H pixels, measured in exact int64 sums
    s.n = whole ? p->width * p->height : s.B * s.B;
    CSV_REQUIRE(whole || s.n <= 2048, CSV_EUNSUPPORTED, "n > 2048 breaks exact FP32 measurement");
    int M = p->m;
    if (M == 0) {
        CSV_REQUIRE(p->rho > 0.f && p->rho <= 1.f, CSV_EINVAL, "rho must be in (0, 1] when m == 0");
        M = (int)std::floor((double)p->rho * s.n + 0.5);
    }
    CSV_REQUIRE(M >= 1 && M <= s.n, CSV_EINVAL, "m must be in [1, n]");
    s.M = M;
    s.Mp = round_up(M, 32);
    s.nbx = whole ? 1 : ceil_div(s.W, s.B);
    s.nby = whole ? 1 : ceil_div(s.H, s.B);
    s.nb = s.nbx * s.nby;
    s.qstep = p->key_qstep;
    s.qshift = 20;
    for (int v = p->key_qstep; v > 1; v >>= 1) ++s.qshift;
    s.T = p->iters;
    s.lambda_frac = p->lambda_frac;
    s.precision = p->precision;
    s.flags = p->flags;
    s.seed = p->phi_seed;
    s.sid = p->stream_id;
    return s;
}

// ------------------------------------------------------------ allocation
void* ctx_alloc(Ctx* c, size_t bytes) {
    if (!bytes) return nullptr;
    CSV_REQUIRE(c->budget == 0 || c->used + bytes <= c->budget, CSV_ENOMEM,
                "context memory budget exceeded (" + std::to_string(c->used + bytes) + " > " +
                    std::to_string(c->budget) + " bytes)");
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{CSV_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
    }
    c->used += bytes;
    return p;
}

void ctx_free(Ctx* c, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    c->used -= bytes;
}

void* scratch(Ctx* c, const std::string& name, size_t bytes) {
    Scratch& s = c->scratch[name];
    if (s.bytes >= bytes) return s.ptr;
    CSV_REQUIRE(!c->capturing, CSV_EINVAL, "scratch would grow during graph capture");
    if (s.ptr) {
        CSV_HIP(hipDeviceSynchronize());   // earlier work may still read the old buffer
        ctx_free(c, s.ptr, s.bytes);
        s.ptr = nullptr;
        s.bytes = 0;
        ++c->gen;   // a buffer moved: graphs captured before now hold stale pointers
    }
    const size_t want = ((bytes + 4095) / 4096) * 4096;
    s.ptr = ctx_alloc(c, want);
    s.bytes = want;
    return s.ptr;
}

static void free_operator(Ctx* c, Operator* op) {
    (void)hipDeviceSynchronize();
    (void)hipFree(op->q);
    c->used -= op->bytes;
}

void free_operators(Ctx* c) {
    if (!c->cache || c->cache.use_count() > 1) return;
    std::lock_guard<std::mutex> lk(c->cache->mu);
    for (auto& kv : c->cache->ops) free_operator(c, kv.second.get());
    c->cache->ops.clear();
}

void release_ctx(Ctx* c) {
    (void)hipDeviceSynchronize();
    free_operators(c);
    for (auto& kv : c->scratch) ctx_free(c, kv.second.ptr, kv.second.bytes);
    c->scratch.clear();
    for (auto& kv : c->beta_tables) (void)hipFree(kv.second.first);
    c->beta_tables.clear();
    if (c->stage_host) (void)hipHostFree(c->stage_host);
    c->stage_host = nullptr;
    if (c->stage_done) (void)hipEventDestroy(c->stage_done);
    c->stage_done = nullptr;
    for (auto& kv : c->prof_pending)
        for (auto& ev : kv.second) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    c->prof_pending.clear();
    for (int i = 0; i < Ctx::kAux; ++i) {
        if (c->aux[i]) (void)hipStreamDestroy(c->aux[i]);
        if (c->aux_done[i]) (void)hipEventDestroy(c->aux_done[i]);
        c->aux[i] = nullptr;
        c->aux_done[i] = nullptr;
    }
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    c->fork_ev = nullptr;
}

using OpKey = std::tuple<uint64_t, uint32_t, int, int, bool>;
static OpKey op_key(const Shape& s) {
    return std::make_tuple(s.seed, s.sid, s.n, s.M, (s.flags & CSV_FLAG_WHOLE_FRAME) != 0);
}

// Build the operator of s into the cache (the cache's lock held).  With
// gram_dst set, a block operator's exact Gram matrix goes there and its
// step constant is left to the caller's batched power iteration.
static Operator* build_operator_locked(Ctx* c, const Shape& s, hipStream_t st,
                                       int* gram_dst = nullptr) {
    const bool whole = (s.flags & CSV_FLAG_WHOLE_FRAME) != 0;
    const OpKey key = op_key(s);
    CSV_REQUIRE(!c->capturing, CSV_EINVAL, "operator setup during graph capture");
    auto op = std::make_unique<Operator>();
    op->B = s.B;
    op->n = s.n;
    op->M = s.M;
    op->Mp = s.Mp;
    op->seed = s.seed;
    op->sid = s.sid;
    op->s_phi = 1.0 / (4.0 * std::sqrt((double)s.M));
    op->whole = whole;
    const size_t n = s.n, Mp = s.Mp;
    if (whole) {
        // Q (Mp x W H int8) for the forward product, Q^T (W H x Mp) for the
        // adjoint, and the step constant; no transform, no FP32 or BF16 copies
        CSV_REQUIRE(s.n % 64 == 0, CSV_EUNSUPPORTED,
                    "whole-frame recovery needs W H to be a multiple of 64");
        const size_t sz_q = (Mp * n + 255) / 256 * 256;
        char* base = static_cast<char*>(ctx_alloc(c, 2 * sz_q + 256));
        op->bytes = 2 * sz_q + 256;
        op->q = reinterpret_cast<int8_t*>(base);
        op->qt = reinterpret_cast<int8_t*>(base + sz_q);
        op->lip = reinterpret_cast<double*>(base + 2 * sz_q);
        try {
            launch_phi_q(op->q, s.M, s.Mp, s.n, s.seed, (uint64_t)s.sid, st);
            launch_transpose_q(op->q, s.Mp, s.n, op->qt, st);
            int* gram = static_cast<int*>(scratch(c, "gram", (size_t)s.M * gram_ld(s.M) * 4));
            void* work = power_work_bytes(s.M) ? scratch(c, "pow_work", power_work_bytes(s.M)) : nullptr;
            launch_power_iteration(op.get(), gram, work, st);
        } catch (...) {
            free_operator(c, op.get());
            throw;
        }
        Operator* raw = op.get();
        c->cache->ops.emplace(key, std::move(op));
        return raw;
    }
    // one allocation, carved into 256-byte aligned pieces
    const size_t sz_q = Mp * n, sz_a64 = Mp * n * 8, sz_a32 = Mp * n * 4;
    const size_t sz_frag = Mp * n * 2, sz_lip = 64, sz_dct = n * 4, sz_dct64 = n * 8;
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t total = 4 * al(sz_q) + al(sz_a64) + 2 * al(sz_a32) + 4 * al(sz_frag) +
                         al(sz_lip) + al(sz_dct) + al(sz_dct64);
    char* base = static_cast<char*>(ctx_alloc(c, total));
    op->bytes = total;
    size_t off = 0;
    auto take = [&](size_t v) {
        char* p = base + off;
        off += al(v);
        return p;
    };
    op->q = reinterpret_cast<int8_t*>(take(sz_q));
    op->q8 = reinterpret_cast<uint8_t*>(take(sz_q));
    op->qb_fwd = reinterpret_cast<uint8_t*>(take(sz_q));
    op->qb_adj = reinterpret_cast<uint8_t*>(take(sz_q));
    op->a64 = reinterpret_cast<double*>(take(sz_a64));
    op->a32 = reinterpret_cast<float*>(take(sz_a32));
    op->phi32 = reinterpret_cast<float*>(take(sz_a32));
    op->frag_fwd = reinterpret_cast<uint16_t*>(take(sz_frag));
    op->frag_adj = reinterpret_cast<uint16_t*>(take(sz_frag));
    op->phi_frag_fwd = reinterpret_cast<uint16_t*>(take(sz_frag));
    op->phi_frag_adj = reinterpret_cast<uint16_t*>(take(sz_frag));
    op->lip = reinterpret_cast<double*>(take(sz_lip));
    op->dct = reinterpret_cast<float*>(take(sz_dct));
    op->dct64 = reinterpret_cast<double*>(take(sz_dct64));
    try {
        launch_phi_q(op->q, s.M, s.Mp, s.n, s.seed, (uint64_t)s.sid, st);
        launch_q_e4m3(op->q, op->q8, s.Mp * s.n, st);
        launch_operator_setup(op.get(), st);
        launch_bf16_frag_layout(op.get(), st);
        launch_q8_frag_layout(op.get(), st);
        if (gram_dst) {
            launch_gram(op.get(), gram_dst, st);
        } else {
            int* gram = static_cast<int*>(scratch(c, "gram", (size_t)s.M * gram_ld(s.M) * 4));
            void* work = power_work_bytes(s.M) ? scratch(c, "pow_work", power_work_bytes(s.M)) : nullptr;
            launch_power_iteration(op.get(), gram, work, st);
        }
    } catch (...) {
        free_operator(c, op.get());
        throw;
    }
    Operator* raw = op.get();
    c->cache->ops.emplace(key, std::move(op));
    return raw;
}

Operator* get_operator(Ctx* c, const Shape& s, hipStream_t st) {
    std::lock_guard<std::mutex> lk(c->cache->mu);
    auto it = c->cache->ops.find(op_key(s));
    if (it != c->cache->ops.end()) return it->second.get();
    return build_operator_locked(c, s, st);
}

void prepare_operators(Ctx* c, const Shape* shapes, int count, hipStream_t st) {
    std::lock_guard<std::mutex> lk(c->cache->mu);
    // the block operators of this call that are not cached yet, once each
    // (whole-frame operators, with their large Gram matrices, are built
    // one at a time by get_operator)
    std::vector<const Shape*> todo;
    std::vector<OpKey> keys;
    for (int i = 0; i < count; ++i) {
        const Shape& s = shapes[i];
        if (s.G < 2 || (s.flags & CSV_FLAG_WHOLE_FRAME)) continue;
        const OpKey k = op_key(s);
        if (c->cache->ops.count(k) || std::find(keys.begin(), keys.end(), k) != keys.end())
            continue;
        keys.push_back(k);
        todo.push_back(&s);
    }
    if (todo.size() < 2) {   // nothing to batch: get_operator builds it when asked
        return;
    }
    std::vector<size_t> off(todo.size() + 1, 0);
    for (size_t i = 0; i < todo.size(); ++i)
        off[i + 1] = off[i] + ((size_t)todo[i]->M * gram_ld(todo[i]->M) + 63) / 64 * 64;
    int* grams = static_cast<int*>(scratch(c, "gram_batch", off.back() * 4));
    std::vector<Operator*> ops;
    std::vector<int*> gp;
    for (size_t i = 0; i < todo.size(); ++i) {
        gp.push_back(grams + off[i]);
        ops.push_back(build_operator_locked(c, *todo[i], st, gp.back()));
    }
    size_t wb = 0;
    for (const Shape* sh : todo) wb = std::max(wb, power_work_bytes(sh->M));
    void* work = wb ? scratch(c, "pow_work", wb) : nullptr;
    launch_power_batch(ops.data(), gp.data(), (int)ops.size(), work, st);
}

// beta_k = (t_k - 1) / t_{k+1}, t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
// (FISTA momentum, Beck and Teboulle 2009), computed in FP64 and stored as
// FP32; all zero for the momentum-free proximal gradient.
const float* beta_table(Ctx* c, int T, bool ista, hipStream_t st) {
    const int key = T * 2 + (ista ? 1 : 0);
    auto it = c->beta_tables.find(key);
    if (it != c->beta_tables.end()) return it->second.first;
    CSV_REQUIRE(!c->capturing, CSV_EINVAL, "momentum table missing during graph capture");
    std::vector<float> h(T);
    double t = 1.0;
    for (int k = 0; k < T; ++k) {
        const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
        h[k] = ista ? 0.f : (float)((t - 1.0) / tn);
        t = tn;
    }
    float* d = static_cast<float*>(ctx_alloc(c, (size_t)T * 4));
    CSV_HIP(hipMemcpyAsync(d, h.data(), (size_t)T * 4, hipMemcpyHostToDevice, st));
    CSV_HIP(hipStreamSynchronize(st));
    c->beta_tables[key] = {d, T};
    return d;
}

// Monotone FISTA (Beck and Teboulle 2009, MFISTA): with the same t_k,
// v_{k+1} = s_k + (t_k / t_{k+1}) (z_k - s_k) + ((t_k - 1) / t_{k+1})
// (s_k - s_{k-1}); the pair (t_k / t_{k+1}, (t_k - 1) / t_{k+1}) per k,
// computed in FP64 and stored as FP32.  Kept under key -T (FISTA and ISTA
// tables use 2 T and 2 T + 1).
const float* mfista_table(Ctx* c, int T, hipStream_t st) {
    const int key = -T;
    auto it = c->beta_tables.find(key);
    if (it != c->beta_tables.end()) return it->second.first;
    CSV_REQUIRE(!c->capturing, CSV_EINVAL, "momentum table missing during graph capture");
    std::vector<float> h(2 * (size_t)T);
    double t = 1.0;
    for (int k = 0; k < T; ++k) {
        const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
        h[2 * k] = (float)(t / tn);
        h[2 * k + 1] = (float)((t - 1.0) / tn);
        t = tn;
    }
    float* d = static_cast<float*>(ctx_alloc(c, h.size() * 4));
    CSV_HIP(hipMemcpyAsync(d, h.data(), h.size() * 4, hipMemcpyHostToDevice, st));
    CSV_HIP(hipStreamSynchronize(st));
    c->beta_tables[key] = {d, 2 * T};
    return d;
}

// --------------------------------------------------------- recovery core
static void lambda_pass(Ctx* c, const Shape& s, Operator* op, const float* y, int nblk, float* lam,
                        hipStream_t st, const std::string& g0name) {
    float* g0 = static_cast<float*>(scratch(c, g0name, (size_t)nblk * s.n * 4));
    F32Batch bt{};
    bt.j[0].op = (s.flags & (CSV_FLAG_LAMBDA_PIXEL_DOMAIN | CSV_FLAG_TV)) ? op->phi32 : op->a32;
    bt.j[0].R = const_cast<float*>(y);   // read only: the adjoint's input
    bt.j[0].G = g0;
    bt.j[0].nblk = nblk;
    launch_f32_adjoint(bt, 1, s.n, s.Mp, st);   // g0 = y^ A (or y^ Phi)
    launch_row_absmax(g0, nblk, s.n, s.n, s.lambda_frac, lam, st);
}

// A GOP of a plain FP32 batch: its operator, dequantised y^, lambda and
// output s (x for TV).
struct F32Item {
    Operator* op;
    const float* y;
    const float* lam;
    float* S;
    int nblk;
};

// Total-variation recovery (k_tv.hip) in FP32, pixel domain, for up to
// kF32Batch GOPs of one shape: the GOPs' images are stacked in xs (their
// rows in item order) so the dual and primal steps run once per group,
// and the two Phi products run batched on FP32 MFMA (R = x Phi^T - y^,
// Gd = R Phi).  xs receives x; the caller points each item at its rows.
static void tv_fp32(Ctx* c, const Shape& s, const std::vector<F32Item>& its, float* xs,
                    hipStream_t st) {
    const int ng = (int)its.size();
    CSV_REQUIRE(ng >= 1 && ng <= kF32Batch, CSV_EINVAL, "FP32 batch size");
    int total = 0;
    for (const F32Item& it : its) total += it.nblk;
    const size_t nn = (size_t)total * s.n;
    float* nuh = static_cast<float*>(scratch(c, "tv_nuh", nn * 4));
    float* nuv = static_cast<float*>(scratch(c, "tv_nuv", nn * 4));
    float* wh = static_cast<float*>(scratch(c, "tv_wh", nn * 4));
    float* wv = static_cast<float*>(scratch(c, "tv_wv", nn * 4));
    float* ph = static_cast<float*>(scratch(c, "tv_ph", nn * 4));
    float* pv = static_cast<float*>(scratch(c, "tv_pv", nn * 4));
    float* Gd = static_cast<float*>(scratch(c, "Gd", nn * 4));
    float* R = static_cast<float*>(scratch(c, "Rm", (size_t)total * s.Mp * 4));
    float* lam = static_cast<float*>(scratch(c, "tv_lam", (size_t)total * 4));
    float* alpha = static_cast<float*>(scratch(c, "tv_alpha", (size_t)total * 4));
    F32Batch bt{};
    size_t off = 0;
    for (int g = 0; g < ng; ++g) {
        const F32Item& it = its[g];
        bt.j[g] = F32Job{it.op->phi32, it.y, it.lam, it.op->lip, nullptr, xs + off * s.n,
                         Gd + off * s.n, R + off * s.Mp, it.nblk};
        launch_copy_f32(lam + off, it.lam, (size_t)it.nblk, st);
        launch_tv_alpha(it.op->lip, it.lam, it.nblk, alpha + off, st);
        off += (size_t)it.nblk;
    }
    for (float* p : {xs, nuh, nuv, wh, wv}) launch_fill_f32(p, 0.f, nn, st);
    for (int k = 0; k < s.T; ++k) {
        launch_tv_dual(xs, nuh, nuv, wh, wv, ph, pv, lam, total, s.B, s.B, st);
        launch_f32_forward(bt, ng, s.n, s.M, s.Mp, st);
        launch_f32_adjoint(bt, ng, s.n, s.Mp, st);
        launch_tv_primal(xs, Gd, ph, pv, alpha, total, s.B, s.B, st);
    }
}

// Plain FP32 FISTA for up to kF32Batch GOPs of one shape (n, M, M_p, T,
// ISTA / monotone), all sharing each launch (k_fp32_mfma.hip).  Each GOP k
// of the batch has its own iterate scratch ("V#k", "Rm#k"; the monotone
// variant adds "Z#k", "AZ#k", "AS#k", "FS#k").
static void mfista_fp32(Ctx* c, const Shape& s, F32Batch& bt, int ng, hipStream_t st);

static void fista_fp32(Ctx* c, const Shape& s, const std::vector<F32Item>& its, hipStream_t st) {
    const int ng = (int)its.size();
    CSV_REQUIRE(ng >= 1 && ng <= kF32Batch, CSV_EINVAL, "FP32 batch size");
    F32Batch bt{};
    for (int g = 0; g < ng; ++g) {
        const F32Item& it = its[g];
        const size_t nn = (size_t)it.nblk * s.n;
        const std::string tag = "#" + std::to_string(g);
        F32Job& j = bt.j[g];
        j.op = it.op->a32;
        j.y = it.y;
        j.lam = it.lam;
        j.lip = it.op->lip;
        j.S = it.S;
        j.V = static_cast<float*>(scratch(c, "V" + tag, nn * 4));
        j.R = static_cast<float*>(scratch(c, "Rm" + tag, (size_t)it.nblk * s.Mp * 4));
        j.nblk = it.nblk;
        if (s.flags & CSV_FLAG_MONOTONE) {
            j.Z = static_cast<float*>(scratch(c, "Z" + tag, nn * 4));
            j.AZ = static_cast<float*>(scratch(c, "AZ" + tag, (size_t)it.nblk * s.Mp * 4));
            j.AS = static_cast<float*>(scratch(c, "AS" + tag, (size_t)it.nblk * s.Mp * 4));
            j.FS = static_cast<double*>(scratch(c, "FS" + tag, (size_t)it.nblk * 8));
        }
    }
    if (s.flags & CSV_FLAG_MONOTONE) {
        mfista_fp32(c, s, bt, ng, st);
        return;
    }
    const float* beta = beta_table(c, s.T, (s.flags & CSV_FLAG_ISTA) != 0, st);
    for (int g = 0; g < ng; ++g) {
        launch_fill_f32(bt.j[g].S, 0.f, (size_t)its[g].nblk * s.n, st);
        launch_fill_f32(bt.j[g].V, 0.f, (size_t)its[g].nblk * s.n, st);
    }
    for (int k = 0; k < s.T; ++k) {
        // residual A v - y^ (padded rows 0); gradient A^T (A v - y^) and the
        // threshold and momentum step in one pass
        launch_f32_forward(bt, ng, s.n, s.M, s.Mp, st);
        launch_f32_adjoint_prox(bt, ng, s.n, s.Mp, beta, k, st);
    }
}

// Monotone FISTA on the batch: per iteration the adjoint with the prox step
// (z_k), the forward product A z_k, and the per-block choice of s_k with the
// extrapolation of v_{k+1}, A s_k and the residual A v_{k+1} - y^.
static void mfista_fp32(Ctx* c, const Shape& s, F32Batch& bt, int ng, hipStream_t st) {
    const float* coef = mfista_table(c, s.T, st);
    F32Batch fz = bt;   // forward product A z_k: X = Z, output AZ, no y^
    for (int g = 0; g < ng; ++g) {
        fz.j[g].V = bt.j[g].Z;
        fz.j[g].R = bt.j[g].AZ;
        fz.j[g].y = nullptr;
    }
    launch_mfista_init(bt, ng, s.n, s.M, s.Mp, st);
    for (int k = 0; k < s.T; ++k) {
        launch_f32_adjoint_zstep(bt, ng, s.n, s.Mp, st);
        launch_f32_forward(fz, ng, s.n, s.M, s.Mp, st);
        launch_mfista_select(bt, ng, s.n, s.M, s.Mp, coef, k, st);
    }
}

static void ensure_aux(Ctx* c);
static void fork_aux(Ctx* c, hipStream_t st);
static void join_aux(Ctx* c, hipStream_t st);

// One recovery job of the fused path: nblk blocks of one operator.
struct FusedJob {
    const Shape* s;
    Operator* op;
    const float* y;
    const float* lam;
    float* S;
    int nblk;
    bool tv = false;   // total-variation recovery (Phi fragments, k_tv_bf16.hip)
};

// Split every job into tiles of 32*CT blocks, group the tiles by (n, Mp)
// class and give each class one persistent launch.  The tile list of a
// class is cut into eight contiguous runs, one per XCD queue (workgroup
// b is dispatched to XCD b % 8), so tiles of one operator stay on few L2s;
// idle workgroups steal from the other queues.
static void fista_bf16(Ctx* c, const std::vector<FusedJob>& jobs, hipStream_t st,
                       int variant = -1) {
    // class key (n, Mp, tv); TV tiles are 32 blocks and use the Phi fragments.
    // The kernel variant of each l1 class is read once, here: the tile width
    // and the launch below both follow that one reading, even if the
    // autotuner changes the process-wide choice meanwhile.
    std::map<std::tuple<int, int, int>, std::vector<FusedTile>> classes;
    std::map<std::pair<int, int>, int> pick;   // (n, Mp) -> variant index
    for (const FusedJob& j : jobs) {
        const Shape& s = *j.s;
        CSV_REQUIRE(!(s.flags & CSV_FLAG_MONOTONE), CSV_EUNSUPPORTED,
                    "monotone FISTA runs on the plain FP32 path only (CSV_FP32)");
        if (j.tv) {
            CSV_REQUIRE(tv_class_supported(s.n, s.Mp), CSV_EUNSUPPORTED,
                        "fused BF16 TV recovery runs on 16 x 16 blocks with M up to 128; "
                        "use CSV_FP32 otherwise");
        } else {
            CSV_REQUIRE(fused_class_supported(s.n, s.Mp), CSV_EUNSUPPORTED,
                        "fused BF16 recovery has no kernel for n=" + std::to_string(s.n) +
                            ", M padded to " + std::to_string(s.Mp));
        }
        int nt = 32;
        if (!j.tv) {
            auto pk = pick.find({s.n, s.Mp});
            if (pk == pick.end())
                pk = pick.emplace(std::make_pair(s.n, s.Mp),
                                  variant >= 0 ? variant : fused_choice(s.n, s.Mp))
                         .first;
            const auto& vs = fused_variants(s.n, s.Mp);
            CSV_REQUIRE(pk->second >= 0 && pk->second < (int)vs.size(), CSV_EINVAL,
                        "no such kernel variant");
            nt = 32 * vs[pk->second].ct;
        }
        const float* beta = beta_table(c, s.T, (s.flags & CSV_FLAG_ISTA) != 0, st);
        for (int b0 = 0; b0 < j.nblk; b0 += nt) {
            FusedTile t{};
            t.frag_fwd = j.tv ? j.op->phi_frag_fwd : j.op->frag_fwd;
            t.frag_adj = j.tv ? j.op->phi_frag_adj : j.op->frag_adj;
            t.qb_fwd = j.op->qb_fwd;
            t.qb_adj = j.op->qb_adj;
            t.dct = j.op->dct;
            t.s_phi = (float)j.op->s_phi;
            t.lip = j.op->lip;
            t.y = j.y + (size_t)b0 * s.Mp;
            t.lam = j.lam + b0;
            t.s = j.S + (size_t)b0 * s.n;
            t.beta = beta;
            t.nblk = std::min(nt, j.nblk - b0);
            t.T = s.T;
            t.n = s.n;
            t.Mp = s.Mp;
            classes[{s.n, s.Mp, j.tv ? 1 : 0}].push_back(t);
        }
    }
    if (classes.empty()) return;
    // host staging: [tiles][qoff 9 + queue + counters 8] per class, one upload
    size_t tiles_bytes = 0, idx_ints = 0;
    for (auto& kv : classes) {
        tiles_bytes += kv.second.size() * sizeof(FusedTile);
        idx_ints += 9 + kv.second.size() + 8;
    }
    const size_t bytes = tiles_bytes + idx_ints * sizeof(int) + 64;
    char* host = nullptr;
    c->last_table_bytes = bytes;
    if (c->capturing) {
        // the graph replays this upload from a buffer nobody else rewrites
        CSV_REQUIRE(c->capture_host && bytes <= c->capture_bytes, CSV_EINVAL,
                    "tile table larger than the capture buffer");
        host = static_cast<char*>(c->capture_host);
    } else {
        if (c->stage_bytes < bytes) {
            if (c->stage_host) {
                CSV_HIP(hipEventSynchronize(c->stage_done));
                CSV_HIP(hipHostFree(c->stage_host));
            }
            c->stage_host = nullptr;
            c->stage_bytes = 0;
            CSV_HIP(hipHostMalloc(&c->stage_host, bytes * 2, hipHostMallocDefault));
            c->stage_bytes = bytes * 2;
        } else if (c->stage_host) {
            CSV_HIP(hipEventSynchronize(c->stage_done));   // previous upload has left the buffer
        }
        if (!c->stage_done) CSV_HIP(hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming));
        host = static_cast<char*>(c->stage_host);
    }
    char* dev = static_cast<char*>(scratch(c, "tiles", bytes));
    struct Launch {
        int n, Mp, tv, count;
        size_t tiles_off, qoff_off, queue_off, ctr_off;
        int variant;
    };
    std::vector<Launch> launches;
    size_t off_t = 0, off_i = tiles_bytes;
    for (auto& kv : classes) {
        const auto& v = kv.second;
        const int count = (int)v.size();
        Launch L{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), count,
                 off_t, 0, 0, 0, -1};
        if (!L.tv) {
            L.variant = pick.at({L.n, L.Mp});
            // every tile must fit the workgroup of the variant that runs it
            const int cap = 32 * fused_variants(L.n, L.Mp)[L.variant].ct;
            for (const FusedTile& t : v)
                CSV_REQUIRE(t.nblk >= 1 && t.nblk <= cap, CSV_EINVAL,
                            "tile wider than the kernel variant's workgroup");
        }
        std::memcpy(host + off_t, v.data(), v.size() * sizeof(FusedTile));
        off_t += v.size() * sizeof(FusedTile);
        int* qoff = reinterpret_cast<int*>(host + off_i);
        L.qoff_off = off_i;
        for (int x = 0; x <= 8; ++x) qoff[x] = (int)((long long)count * x / 8);
        off_i += 9 * sizeof(int);
        int* queue = reinterpret_cast<int*>(host + off_i);
        L.queue_off = off_i;
        for (int i = 0; i < count; ++i) queue[i] = i;
        off_i += count * sizeof(int);
        int* ctr = reinterpret_cast<int*>(host + off_i);
        L.ctr_off = off_i;
        for (int x = 0; x < 8; ++x) ctr[x] = 0;
        off_i += 8 * sizeof(int);
        launches.push_back(L);
    }
    CSV_HIP(hipMemcpyAsync(dev, host, off_i, hipMemcpyHostToDevice, st));
    if (!c->capturing) CSV_HIP(hipEventRecord(c->stage_done, st));
    // several classes run side by side: largest first, round-robin over st
    // and the auxiliary streams, so small classes fill the CUs that a large
    // class leaves idle (each class has its own queues; no workgroup waits
    // for another)
    std::sort(launches.begin(), launches.end(), [](const Launch& a, const Launch& b) {
        return (double)a.count * a.n * a.Mp > (double)b.count * b.n * b.Mp;
    });
    const bool spread = launches.size() > 1;
    if (spread) {
        ensure_aux(c);
        fork_aux(c, st);
    }
    for (size_t k = 0; k < launches.size(); ++k) {
        const Launch& L = launches[k];
        const int lane = (int)(k % (Ctx::kAux + 1));
        const hipStream_t ls = lane == 0 ? st : c->aux[lane - 1];
        const auto* tiles = reinterpret_cast<const FusedTile*>(dev + L.tiles_off);
        const auto* qoff = reinterpret_cast<const int*>(dev + L.qoff_off);
        const auto* queue = reinterpret_cast<const int*>(dev + L.queue_off);
        auto* ctr = reinterpret_cast<int*>(dev + L.ctr_off);
        if (L.tv) {
            ProfScope ps(c, "tv_bf16", ls);
            launch_tv_bf16_class(L.n, L.Mp, tiles, qoff, queue, ctr, L.count, device_cus(), ls);
        } else {
            ProfScope ps(c, "fista_bf16", ls);
            launch_fista_bf16_class(L.n, L.Mp, tiles, qoff, queue, ctr, L.count, ls, L.variant);
        }
    }
    if (spread) join_aux(c, st);
}

// Time one fused launch over nblk blocks with kernel variant `variant`
// (milliseconds, HIP events on `st`, median of `reps`).
double time_fused_variant(Ctx* c, const Shape& s, Operator* op, const float* y, const float* lam,
                          float* S, int nblk, int variant, int reps, hipStream_t st) {
    std::vector<FusedJob> jobs{FusedJob{&s, op, y, lam, S, nblk}};
    fista_bf16(c, jobs, st, variant);   // warm-up (also sets the kernel attributes)
    hipEvent_t a, b;
    CSV_HIP(hipEventCreate(&a));
    CSV_HIP(hipEventCreate(&b));
    std::vector<double> ms;
    for (int r = 0; r < reps; ++r) {
        CSV_HIP(hipEventRecord(a, st));
        fista_bf16(c, jobs, st, variant);
        CSV_HIP(hipEventRecord(b, st));
        CSV_HIP(hipEventSynchronize(b));
        float t = 0.f;
        CSV_HIP(hipEventElapsedTime(&t, a, b));
        ms.push_back(t);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::sort(ms.begin(), ms.end());
    return ms[ms.size() / 2];
}

// Dequantise and compute lambda for nblk blocks of one operator; returns y^.
const float* prepare(Ctx* c, const Shape& s, Operator* op, const int8_t* codes,
                            const uint8_t* exps, int nblk, float* lam, const std::string& tag,
                            hipStream_t st, const std::string& g0name) {
    float* y = static_cast<float*>(scratch(c, "yhat" + tag, (size_t)nblk * s.Mp * 4));
    launch_dequant(codes, exps, nblk, s.M, s.Mp, op->s_phi, y, st,
                   (s.flags & CSV_FLAG_NO_QUANT) != 0);
    lambda_pass(c, s, op, y, nblk, lam, st, g0name);
    return y;
}

void recover(Ctx* c, const Shape& s, Operator* op, const int8_t* codes, const uint8_t* exps,
             int nblk, float* S, float* lam_out, double* obj_out, hipStream_t st) {
    if (nblk <= 0) return;
    float* lam = lam_out ? lam_out : static_cast<float*>(scratch(c, "lam", (size_t)nblk * 4));
    const bool tv = (s.flags & CSV_FLAG_TV) != 0;
    const float* y = prepare(c, s, op, codes, exps, nblk, lam, "", st);
    if (tv && s.precision == CSV_FP32) {
        ProfScope ps(c, "tv_fp32", st);
        tv_fp32(c, s, {F32Item{op, y, lam, S, nblk}}, S, st);
    } else if (tv) {
        FusedJob j{&s, op, y, lam, S, nblk};
        j.tv = true;
        fista_bf16(c, {j}, st);
    } else if (s.precision == CSV_FP32) {
        ProfScope ps(c, "fista_fp32", st);
        fista_fp32(c, s, {F32Item{op, y, lam, S, nblk}}, st);
    } else {
        fista_bf16(c, {FusedJob{&s, op, y, lam, S, nblk}}, st);
    }
    if (obj_out) {
        ProfScope ps(c, "final64", st);
        if (tv)
            launch_tv_final64(op->q, S, codes, exps, lam, nblk, s.M, s.B, op->s_phi, obj_out, st);
        else
            launch_final64(op->a64, S, codes, exps, lam, nblk, s.M, s.Mp, s.n, op->s_phi,
                           obj_out, st, (s.flags & CSV_FLAG_NO_QUANT) != 0);
    }
}

// Event-timed ranges of named kernels on the stream they are launched on.
ProfScope::ProfScope(Ctx* c, const char* name, hipStream_t st) : c_(c), name_(name), st_(st) {
    if (!c_->profiling) return;
    CSV_HIP(hipEventCreate(&a_));
    CSV_HIP(hipEventCreate(&b_));
    CSV_HIP(hipEventRecord(a_, st_));
}

ProfScope::~ProfScope() {
    if (!c_->profiling || !a_) return;
    if (hipEventRecord(b_, st_) == hipSuccess) c_->prof_pending[name_].push_back({a_, b_});
}

// Decode `count` GOPs.  Key frames first (Section 3.2: CS frames are decoded
// only after the key frame), then one recovery pass over every CS block of
// every GOP, then synthesis onto each decoded key frame (eq. (4)).
// Forward declarations of the batch helpers below.
static void ensure_aux(Ctx* c);
static void fork_aux(Ctx* c, hipStream_t st);
static void join_aux(Ctx* c, hipStream_t st);

// Lane k of the per-GOP chains: 0 is st itself, 1..kAux the auxiliary
// streams, so that st and the kAux streams fill the process's hardware queues
// while the chains run side by side.
static hipStream_t chain_lane(Ctx* c, hipStream_t st, int k) {
    return k == 0 ? st : c->aux[k - 1];
}

// Encode `count` GOPs (Section 3.1, Fig. 3): key frame coded and decoded,
// every CS frame's residual against the decoded key frame (eqs. (2)-(3))
// measured per block and quantised.  GOP i runs on lane i % (kAux + 1) with
// scratch of its own (one GOP alone runs on st).
void encode_gops(Ctx* c, int count, const Shape* shapes, const uint8_t* const* frames,
                 const csv_gop_stream* out, hipStream_t st) {
    std::vector<Operator*> ops(count, nullptr);
    prepare_operators(c, shapes, count, st);   // new streams' setup in one batch
    for (int i = 0; i < count; ++i) {
        const Shape& s = shapes[i];
        CSV_REQUIRE(frames[i] && out[i].key_levels, CSV_EINVAL, "NULL frames or key_levels");
        CSV_REQUIRE(s.G == 1 || (out[i].codes && out[i].exps), CSV_EINVAL, "codes/exps are NULL");
        if (s.G > 1 && !(s.flags & CSV_FLAG_WHOLE_FRAME)) ops[i] = get_operator(c, s, st);
    }
    const bool spread = count > 1;
    if (spread) ensure_aux(c);
    std::vector<uint8_t*> keydec(count, nullptr);
    std::vector<int32_t*> ymeas(count, nullptr);
    for (int i = 0; i < count; ++i) {   // scratch is sized before any launch
        const Shape& s = shapes[i];
        if (s.G == 1) continue;
        const std::string tag = spread ? "#" + std::to_string(i) : std::string();
        keydec[i] = static_cast<uint8_t*>(scratch(c, "keydec" + tag, (size_t)s.W * s.H));
        // int32 per padded row, or int64 per row for whole frames
        ymeas[i] = static_cast<int32_t*>(
            scratch(c, "ymeas" + tag, (size_t)(s.G - 1) * s.nb * s.Mp * 8));
    }
    if (spread) fork_aux(c, st);
    for (int i = 0; i < count; ++i) {
        const Shape& s = shapes[i];
        const hipStream_t ls = spread ? chain_lane(c, st, i % (Ctx::kAux + 1)) : st;
        const int ncs = s.G - 1;
        unsigned long long* bits = reinterpret_cast<unsigned long long*>(out[i].bits);
        if (bits) {
            launch_fill_u64(bits, 0ull, 1, ls);
            const bool raw = (s.flags & CSV_FLAG_NO_QUANT) != 0;
            launch_fill_u64(bits + 1,
                            (unsigned long long)ncs * s.nb * (raw ? 32ull * s.M : 8ull * s.M + 8ull),
                            1, ls);
        }
        launch_key_encode(frames[i], s.W, s.H, s.qshift, out[i].key_levels, bits, ls);
        if (!ncs) continue;
        launch_key_decode(out[i].key_levels, s.W, s.H, s.qstep, keydec[i], ls);
        const size_t fs = (size_t)s.W * s.H;
        const int total = ncs * s.nb;
        if (s.flags & CSV_FLAG_WHOLE_FRAME) {
            long long* y64 = reinterpret_cast<long long*>(ymeas[i]);
            {
                ProfScope ps(c, "measure", ls);
                launch_whole_measure(s, frames[i] + fs, ncs, fs, keydec[i], y64, ls);
            }
            launch_whole_quantise(y64, s.M, ncs, out[i].codes, out[i].exps, nullptr, ls);
            continue;
        }
        {
            ProfScope ps(c, "measure", ls);
            launch_measure(s, ops[i]->q, ops[i]->q8, frames[i] + fs, ncs, fs, keydec[i], ymeas[i],
                           ls);
        }
        launch_quantise(ymeas[i], s.M, s.Mp, total, out[i].codes, out[i].exps, nullptr, ls,
                        (s.flags & CSV_FLAG_NO_QUANT) != 0);
    }
    if (spread) join_aux(c, st);
}

// Fork: the auxiliary streams wait for everything enqueued on st so far.
// Join: st waits for everything enqueued on the auxiliary streams.  Both are
// event edges, so they also hold inside a stream capture.
static void ensure_aux(Ctx* c) {
    if (c->fork_ev) return;
    CSV_REQUIRE(!c->capturing, CSV_EINVAL, "auxiliary streams created during graph capture");
    for (int i = 0; i < Ctx::kAux; ++i) {
        CSV_HIP(hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking));
        CSV_HIP(hipEventCreateWithFlags(&c->aux_done[i], hipEventDisableTiming));
    }
    CSV_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
}

static void fork_aux(Ctx* c, hipStream_t st) {
    CSV_HIP(hipEventRecord(c->fork_ev, st));
    for (int i = 0; i < Ctx::kAux; ++i) CSV_HIP(hipStreamWaitEvent(c->aux[i], c->fork_ev, 0));
}

static void join_aux(Ctx* c, hipStream_t st) {
    for (int i = 0; i < Ctx::kAux; ++i) {
        CSV_HIP(hipEventRecord(c->aux_done[i], c->aux[i]));
        CSV_HIP(hipStreamWaitEvent(st, c->aux_done[i], 0));
    }
}

// Whole-frame recovery (eq. (1) with the TV solver): every CS frame of a
// GOP is one H x W image measured by Phi = s_Phi Q (M x W H).  FP32
// iterates, products with the resident int8 Q in fixed-order partial sums,
// the same dual and primal steps as the block TV solver, FP64 objective per
// frame.  A group of GOPs of one shape (at most kWholeBatch) shares every
// launch of the iteration: the images are [GOP][frame] rows.
struct WholeItem {
    Operator* op;
    const csv_gop_stream* in;
    uint8_t* frames;
    float* cs_float;
    double* obj;
};

static void decode_whole(Ctx* c, const Shape& s, const std::vector<WholeItem>& its,
                         hipStream_t st) {
    const int ng = (int)its.size();
    CSV_REQUIRE(ng >= 1 && ng <= kWholeBatch, CSV_EINVAL, "whole-frame group size");
    {
        ProfScope ps(c, "key_decode", st);
        for (const WholeItem& w : its)
            launch_key_decode(w.in->key_levels, s.W, s.H, s.qstep, w.frames, st);
    }
    const int F = s.G - 1, n = s.n, M = s.M;
    if (F <= 0) return;
    const int nimg = ng * F;
    const size_t nn = (size_t)nimg * n, fm = (size_t)nimg * M;
    const int nk = whole_fwd_parts(n);
    float* y = static_cast<float*>(scratch(c, "w_y", fm * 4));
    float* r = static_cast<float*>(scratch(c, "w_r", fm * 4));
    float* pf = static_cast<float*>(scratch(c, "w_pf", (size_t)nk * fm * 4));
    float* lam = static_cast<float*>(scratch(c, "w_lam", (size_t)nimg * 4));
    float* alpha = static_cast<float*>(scratch(c, "w_alpha", (size_t)nimg * 4));
    float* x = static_cast<float*>(scratch(c, "w_x", nn * 4));
    WholeTv tv{x,
               static_cast<float*>(scratch(c, "tv_nuh", nn * 4)),
               static_cast<float*>(scratch(c, "tv_nuv", nn * 4)),
               static_cast<float*>(scratch(c, "tv_wh", nn * 4)),
               static_cast<float*>(scratch(c, "tv_wv", nn * 4)),
               static_cast<float*>(scratch(c, "tv_ph", nn * 4)),
               static_cast<float*>(scratch(c, "tv_pv", nn * 4)),
               lam,
               alpha};
    bool any_obj = false;
    for (const WholeItem& w : its) any_obj = any_obj || w.obj;
    double* rr = any_obj ? static_cast<double*>(scratch(c, "w_rr", (size_t)F * M * 8)) : nullptr;
    double* yy = any_obj ? static_cast<double*>(scratch(c, "w_yy", (size_t)F * M * 8)) : nullptr;
    WholeQ qs{}, qts{};
    WholeLip ls{};
    for (int g = 0; g < ng; ++g) {
        qs.q[g] = its[g].op->q;
        qts.q[g] = its[g].op->qt;
        ls.lip[g] = its[g].op->lip;
    }
    const double s_phi = its[0].op->s_phi;
    const float sphi = (float)s_phi;
    const WholeTv plain{};
    {
        ProfScope ps(c, "prepare", st);
        for (int g = 0; g < ng; ++g)
            launch_dequant(its[g].in->codes, its[g].in->exps, F, M, M, s_phi,
                           y + (size_t)g * F * M, st);
        // lam = frac ||Phi^T y^||_inf per frame, then the step per frame
        launch_whole_adj(qts, ng, y, F, s.H, s.W, M, s.Mp, sphi, x, plain, st);
        launch_row_absmax(x, nimg, n, n, s.lambda_frac, lam, st);
        launch_whole_alpha(ls, lam, F, ng, alpha, st);
    }
    {
        // per iteration: forward product with the dual step (x -> nu, w, P
        // and the partials), the partials' sum (r), adjoint with the primal
        // step (x); x, nu, w start at zero
        ProfScope ps(c, "tv_whole", st);
        for (float* p : {x, tv.nuh, tv.nuv, tv.wh, tv.wv}) launch_fill_f32(p, 0.f, nn, st);
        for (int k = 0; k < s.T; ++k) {
            launch_whole_fwd(qs, ng, x, F, s.H, s.W, M, sphi, y, pf, r, tv, st);
            launch_whole_adj(qts, ng, r, F, s.H, s.W, M, s.Mp, sphi, nullptr, tv, st);
        }
    }
    for (int g = 0; g < ng; ++g) {
        const WholeItem& w = its[g];
        const float* xg = x + (size_t)g * F * n;
        if (w.obj) {
            ProfScope ps(c, "final64", st);
            launch_whole_objective(w.op->q, xg, F, s.H, s.W, M, s_phi, w.in->codes, w.in->exps,
                                   lam + (size_t)g * F, rr, yy, w.obj, st);
        }
        ProfScope ps(c, "synth", st);
        launch_whole_place(xg, w.frames, F, n, w.frames + n, w.cs_float, st);
    }
}

void decode_gops(Ctx* c, int count, const Shape* shapes, const csv_gop_stream* in,
                 uint8_t* const* frames_out, float* const* cs_float_out, double* const* obj_out,
                 hipStream_t st) {
    struct Item {
        Operator* op = nullptr;
        bool whole = false;
        int nblk = 0;
        float* S = nullptr;
        float* lam = nullptr;
        const float* y = nullptr;
    };
    std::vector<Item> items(count);
    prepare_operators(c, shapes, count, st);   // new streams' setup in one batch
    for (int i = 0; i < count; ++i) {
        const Shape& s = shapes[i];
        CSV_REQUIRE(in[i].key_levels && frames_out[i], CSV_EINVAL, "NULL key_levels or frames_out");
        CSV_REQUIRE(!(s.flags & CSV_FLAG_TV) || s.precision == CSV_FP32 ||
                        tv_class_supported(s.n, s.Mp),
                    CSV_EUNSUPPORTED,
                    "BF16 TV recovery runs on 16 x 16 blocks with M up to 128; use CSV_FP32");
        CSV_REQUIRE(!(s.flags & CSV_FLAG_WHOLE_FRAME) ||
                        ((s.flags & CSV_FLAG_TV) && s.precision == CSV_FP32),
                    CSV_EUNSUPPORTED,
                    "whole-frame measurements are recovered by TV in FP32 only "
                    "(CSV_FLAG_TV, CSV_FP32)");
        CSV_REQUIRE(s.G == 1 || (in[i].codes && in[i].exps), CSV_EINVAL, "codes/exps are NULL");
        CSV_REQUIRE(!(s.flags & CSV_FLAG_MONOTONE) || s.precision == CSV_FP32, CSV_EUNSUPPORTED,
                    "monotone FISTA runs on the plain FP32 path only (CSV_FP32)");
        items[i].op = s.G > 1 ? get_operator(c, s, st) : nullptr;
        items[i].nblk = (s.G - 1) * s.nb;
    }
    // whole-frame GOPs: grouped by shape (frame size, M, G, T, lambda_frac),
    // each group's iterations batched on st (their scratch is the context's)
    bool any_block = false;
    std::map<std::tuple<int, int, int, int, int, float>, std::vector<int>> groups;
    for (int i = 0; i < count; ++i) {
        const Shape& s = shapes[i];
        if (!(s.flags & CSV_FLAG_WHOLE_FRAME)) {
            any_block = true;
            continue;
        }
        groups[std::make_tuple(s.W, s.H, s.M, s.G, s.T, s.lambda_frac)].push_back(i);
        items[i].whole = true;
        items[i].nblk = 0;   // nothing left for the block passes below
    }
    for (const auto& kv : groups) {
        const std::vector<int>& idx = kv.second;
        for (size_t a = 0; a < idx.size(); a += kWholeBatch) {
            std::vector<WholeItem> its;
            for (size_t b = a; b < idx.size() && b < a + kWholeBatch; ++b) {
                const int i = idx[b];
                its.push_back(WholeItem{items[i].op, &in[i], frames_out[i],
                                        cs_float_out ? cs_float_out[i] : nullptr,
                                        obj_out ? obj_out[i] : nullptr});
            }
            decode_whole(c, shapes[idx[a]], its, st);
        }
    }
    if (!any_block) return;
    // GOP i's preparation runs on lane i % (kAux + 1), st included, and its
    // synthesis on auxiliary stream i % kAux, beside the FP64 checks on st
    // (one GOP alone stays on st); each lane has its own lambda scratch
    const bool spread = count > 1;
    if (spread) ensure_aux(c);
    constexpr int kLanes = Ctx::kAux + 1;
    auto prep_lane = [&](int i) { return spread ? chain_lane(c, st, i % kLanes) : st; };
    auto lane_of = [&](int i) { return spread ? c->aux[i % Ctx::kAux] : st; };
    auto g0_of = [&](int i) {
        return spread ? "g0@" + std::to_string(i % kLanes) : std::string("g0");
    };
    // scratch is sized before any launch that reads it
    for (int i = 0; i < count; ++i) {
        const Shape& s = shapes[i];
        if (!items[i].nblk) continue;
        const std::string tag = "#" + std::to_string(i);
        // FP32 TV GOPs get rows of their batch's stacked image buffer later
        if (!(s.precision == CSV_FP32 && (s.flags & CSV_FLAG_TV)))
            items[i].S = static_cast<float*>(scratch(c, "S" + tag, (size_t)items[i].nblk * s.n * 4));
        items[i].lam = static_cast<float*>(scratch(c, "lam" + tag, (size_t)items[i].nblk * 4));
        scratch(c, "yhat" + tag, (size_t)items[i].nblk * s.Mp * 4);
        scratch(c, g0_of(i), (size_t)items[i].nblk * s.n * 4);
    }
    if (spread) fork_aux(c, st);
    for (int i = 0; i < count; ++i) {
        const Shape& s = shapes[i];
        Item& it = items[i];
        const hipStream_t ls = prep_lane(i);
        if (it.whole) continue;
        {
            ProfScope ps(c, "key_decode", ls);
            launch_key_decode(in[i].key_levels, s.W, s.H, s.qstep, frames_out[i], ls);
        }
        if (!it.nblk) continue;
        ProfScope ps(c, "prepare", ls);
        it.y = prepare(c, s, it.op, in[i].codes, in[i].exps, it.nblk, it.lam,
                       "#" + std::to_string(i), ls, g0_of(i));
    }
    if (spread) join_aux(c, st);
    std::vector<FusedJob> jobs;
    // plain FP32 GOPs (l1 and TV): grouped by shape and solver, each group's
    // launches shared
    std::map<std::tuple<int, int, int, int, int, int>, std::vector<int>> f32_groups;
    for (int i = 0; i < count; ++i) {
        const Shape& s = shapes[i];
        Item& it = items[i];
        if (!it.nblk) continue;
        if (s.precision == CSV_FP32) {
            const int tv = (s.flags & CSV_FLAG_TV) ? 1 : 0;
            f32_groups[std::make_tuple(tv, s.n, s.M, s.Mp, s.T,
                                       s.flags & (CSV_FLAG_ISTA | CSV_FLAG_MONOTONE))]
                .push_back(i);
            continue;
        }
        if (s.flags & CSV_FLAG_TV) {
            FusedJob j{&shapes[i], it.op, it.y, it.lam, it.S, it.nblk};
            j.tv = true;
            jobs.push_back(j);
        } else {
            jobs.push_back(FusedJob{&shapes[i], it.op, it.y, it.lam, it.S, it.nblk});
        }
    }
    int tv_batches = 0;   // names each TV batch's stacked image buffer
    for (const auto& kv : f32_groups) {
        const std::vector<int>& idx = kv.second;
        const bool tv = std::get<0>(kv.first) != 0;
        for (size_t a = 0; a < idx.size(); a += kF32Batch) {
            std::vector<F32Item> its;
            std::vector<int> members;
            int total = 0;
            for (size_t b = a; b < idx.size() && b < a + kF32Batch; ++b) {
                const Item& it = items[idx[b]];
                its.push_back(F32Item{it.op, it.y, it.lam, it.S, it.nblk});
                members.push_back(idx[b]);
                total += it.nblk;
            }
            const Shape& s0 = shapes[idx[a]];
            if (tv) {
                // the batch's images stacked in one buffer; each GOP's S
                // then points at its rows (synthesis and the FP64 check
                // read them there)
                ProfScope ps(c, "tv_fp32", st);
                const std::string xname = "tv_x@" + std::to_string(tv_batches++);
                float* xs = static_cast<float*>(scratch(c, xname, (size_t)total * s0.n * 4));
                tv_fp32(c, s0, its, xs, st);
                size_t off = 0;
                for (int i : members) {
                    items[i].S = xs + off * s0.n;
                    off += (size_t)items[i].nblk;
                }
            } else {
                // the context's FP32 scratch: one batch at a time
                ProfScope ps(c, "fista_fp32", st);
                fista_fp32(c, s0, its, st);
            }
        }
    }
    if (!jobs.empty()) fista_bf16(c, jobs, st);
    if (spread) fork_aux(c, st);
    if (obj_out) {
        // FP64 checks of the DCT-l1 GOPs: one launch per (n, M, Mp) group of up
        // to kF64Batch on the launch stream, beside the syntheses on the lanes
        std::map<std::tuple<int, int, int>, std::vector<int>> groups;
        for (int i = 0; i < count; ++i)
            if (items[i].nblk && obj_out[i] && !(shapes[i].flags & CSV_FLAG_TV))
                groups[{shapes[i].n, shapes[i].M, shapes[i].Mp}].push_back(i);
        for (const auto& kv : groups) {
            const std::vector<int>& mem = kv.second;
            for (size_t g0 = 0; g0 < mem.size(); g0 += kF64Batch) {
                F64Batch bt{};
                int ng = 0;
                for (size_t k = g0; k < mem.size() && ng < kF64Batch; ++k) {
                    const int i = mem[k];
                    const Item& it = items[i];
                    bt.j[ng++] = F64Job{it.op->a64, it.S,   in[i].codes,      in[i].exps,
                                        it.lam,     obj_out[i], it.op->s_phi, it.nblk,
                                        (shapes[i].flags & CSV_FLAG_NO_QUANT) ? 1 : 0};
                }
                const Shape& s0 = shapes[mem[g0]];
                ProfScope ps(c, "final64", st);
                launch_final64_batch(bt, ng, s0.M, s0.Mp, s0.n, st);
            }
        }
    }
    for (int i = 0; i < count; ++i) {
        const Shape& s = shapes[i];
        const Item& it = items[i];
        if (!it.nblk) continue;
        const hipStream_t ls = lane_of(i);
        const bool tv = (s.flags & CSV_FLAG_TV) != 0;
        if (obj_out && obj_out[i] && tv) {
            ProfScope ps(c, "final64", ls);
            launch_tv_final64(it.op->q, it.S, in[i].codes, in[i].exps, it.lam, it.nblk, s.M, s.B,
                              it.op->s_phi, obj_out[i], ls);
        }
        ProfScope ps(c, "synth", ls);
        const size_t fs = (size_t)s.W * s.H;
        // TV recovers pixel-domain residuals: no basis to synthesise
        launch_synth(it.S, tv ? nullptr : it.op->dct, frames_out[i], s.W, s.H, s.B, s.nbx, s.nb,
                     s.G - 1, frames_out[i] + fs, cs_float_out ? cs_float_out[i] : nullptr, ls);
    }
    if (spread) join_aux(c, st);
}

}  // namespace csv

using namespace csv;


static Ctx* C(csv_ctx* c) { return &c->impl; }

static void set_device(csv_ctx* ctx) { CSV_HIP(hipSetDevice(ctx->impl.device)); }

extern "C" {

const char* csv_last_error(void) { return g_last_error.c_str(); }

const char* csv_version(void) { return "csv 0.1 gfx950"; }

int csv_create(csv_ctx** out, int device, size_t mem_budget) {
    return guarded([&] {
        CSV_REQUIRE(out != nullptr, CSV_EINVAL, "out is NULL");
        int count = 0;
        CSV_HIP(hipGetDeviceCount(&count));
        CSV_REQUIRE(device >= 0 && device < count, CSV_EINVAL, "no such device");
        CSV_HIP(hipSetDevice(device));
        noalloc_setup(device);   // the allocation-free entry point's array, once per device
        auto* c = new csv_ctx();
        c->impl.device = device;
        c->impl.budget = mem_budget;
        *out = c;
    });
}

int csv_destroy(csv_ctx* ctx) {
    if (!ctx) return CSV_OK;
    return guarded([&] {
        set_device(ctx);
        CSV_HIP(hipDeviceSynchronize());
        release_ctx(&ctx->impl);
        delete ctx;
    });
}

int csv_ctx_bytes(const csv_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return fail(CSV_EINVAL, "NULL argument");
    *bytes = ctx->impl.used;
    return CSV_OK;
}

int csv_params_default(csv_params* p) {
    if (!p) return fail(CSV_EINVAL, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->width = 176;
    p->height = 144;
    p->gop = 4;
    p->block = 16;
    p->m = 0;
    p->rho = 0.25f;
    p->key_qstep = 16;
    p->iters = 300;
    p->lambda_frac = 0.01f;
    p->precision = CSV_BF16;
    return CSV_OK;
}

int csv_resolve(const csv_params* p, int32_t* m, int32_t* blocks_per_frame) {
    return guarded([&] {
        const Shape s = resolve(p);
        if (m) *m = s.M;
        if (blocks_per_frame) *blocks_per_frame = s.nb;
    });
}

int csv_encoded_size(const csv_params* p, size_t* key_elems, size_t* code_bytes,
                     size_t* exp_bytes, uint64_t* bits_cs) {
    return guarded([&] {
        const Shape s = resolve(p);
        const bool raw = (s.flags & CSV_FLAG_NO_QUANT) != 0;   // int32 y~, no exponent
        if (key_elems) *key_elems = (size_t)s.W * s.H;
        if (code_bytes) *code_bytes = (size_t)(s.G - 1) * s.nb * s.M * (raw ? 4 : 1);
        if (exp_bytes) *exp_bytes = (size_t)(s.G - 1) * s.nb;
        if (bits_cs)
            *bits_cs = (uint64_t)(s.G - 1) * s.nb * (raw ? 32ull * s.M : 8ull * s.M + 8ull);
    });
}

int csv_compression_ratio(const csv_params* p, uint64_t bits_key, uint64_t bits_cs, double* total,
                          double* key, double* cs) {
    return guarded([&] {
        const Shape s = resolve(p);
        CSV_REQUIRE(bits_key + bits_cs > 0, CSV_EINVAL, "zero coded bits");
        const double raw = 8.0 * s.W * s.H;
        if (total) *total = s.G * raw / (double)(bits_key + bits_cs);
        if (key) *key = bits_key ? raw / (double)bits_key : INFINITY;
        if (cs) *cs = bits_cs ? (s.G - 1) * raw / (double)bits_cs : INFINITY;
    });
}

int csv_encode_gop(csv_ctx* ctx, const csv_params* p, const uint8_t* frames,
                   const csv_gop_stream* out, void* stream) {
    return guarded([&] {
        CSV_REQUIRE(ctx && frames && out, CSV_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        const Shape s = resolve(p);
        encode_gops(C(ctx), 1, &s, &frames, out, static_cast<hipStream_t>(stream));
    });
}

int csv_encode_batch(csv_ctx* ctx, int32_t count, const csv_params* params,
                     const uint8_t* const* frames, const csv_gop_stream* out, void* stream) {
    return guarded([&] {
        CSV_REQUIRE(count >= 0, CSV_EINVAL, "negative count");
        if (count == 0) return;
        CSV_REQUIRE(ctx && params && frames && out, CSV_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        std::vector<Shape> shapes;
        for (int i = 0; i < count; ++i) shapes.push_back(resolve(&params[i]));
        encode_gops(C(ctx), count, shapes.data(), frames, out, static_cast<hipStream_t>(stream));
    });
}

int csv_decode_gop(csv_ctx* ctx, const csv_params* p, const csv_gop_stream* in,
                   uint8_t* frames_out, float* cs_float_out, double* obj_out, void* stream) {
    return guarded([&] {
        CSV_REQUIRE(ctx && in && frames_out, CSV_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        const Shape s = resolve(p);
        decode_gops(C(ctx), 1, &s, in, &frames_out, &cs_float_out, &obj_out,
                    static_cast<hipStream_t>(stream));
    });
}

int csv_decode_batch(csv_ctx* ctx, int32_t count, const csv_params* params,
                     const csv_gop_stream* in, uint8_t* const* frames_out,
                     float* const* cs_float_out, double* const* obj_out, void* stream) {
    return guarded([&] {
        CSV_REQUIRE(count >= 0, CSV_EINVAL, "negative count");
        if (count == 0) return;
        CSV_REQUIRE(ctx && params && in && frames_out, CSV_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        std::vector<Shape> shapes;
        for (int i = 0; i < count; ++i) shapes.push_back(resolve(&params[i]));
        for (int i = 1; i < count; ++i)
            CSV_REQUIRE(shapes[i].precision == shapes[0].precision, CSV_EINVAL,
                        "one precision per batch");
        decode_gops(C(ctx), count, shapes.data(), in, frames_out, cs_float_out, obj_out,
                    static_cast<hipStream_t>(stream));
    });
}

struct csv_graph {
    csv_ctx* ctx;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void*> keep;   // pinned tile tables the graph uploads from
    int gen = 0;               // the context's scratch generation at capture
};

int csv_graph_capture(csv_ctx* ctx, int32_t count, const csv_params* params,
                      const csv_gop_stream* in, uint8_t* const* frames_out,
                      float* const* cs_float_out, double* const* obj_out, void* stream,
                      csv_graph** out) {
    return guarded([&] {
        CSV_REQUIRE(ctx && params && in && frames_out && out && count > 0, CSV_EINVAL,
                    "NULL argument or empty batch");
        CSV_REQUIRE(stream != nullptr, CSV_EINVAL, "graph capture needs a non-default stream");
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        hipStream_t st = static_cast<hipStream_t>(stream);
        Ctx* c = C(ctx);
        std::vector<Shape> shapes;
        for (int i = 0; i < count; ++i) shapes.push_back(resolve(&params[i]));
        for (int i = 1; i < count; ++i)
            CSV_REQUIRE(shapes[i].precision == shapes[0].precision, CSV_EINVAL,
                        "one precision per batch");
        // eager pass: builds operators, momentum tables and scratch
        decode_gops(c, count, shapes.data(), in, frames_out, cs_float_out, obj_out, st);
        CSV_HIP(hipStreamSynchronize(st));
        auto g = std::make_unique<csv_graph>();
        g->ctx = ctx;
        const bool prof = c->profiling;
        if (c->last_table_bytes) {
            void* keep = nullptr;
            CSV_HIP(hipHostMalloc(&keep, c->last_table_bytes, hipHostMallocDefault));
            g->keep.push_back(keep);
            c->capture_host = keep;
            c->capture_bytes = c->last_table_bytes;
        }
        c->profiling = false;
        c->capturing = true;
        hipError_t cap = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (cap == hipSuccess) {
            try {
                decode_gops(c, count, shapes.data(), in, frames_out, cs_float_out, obj_out, st);
            } catch (...) {
                hipGraph_t junk = nullptr;
                (void)hipStreamEndCapture(st, &junk);
                if (junk) (void)hipGraphDestroy(junk);
                c->capturing = false;
                c->capture_host = nullptr;
                c->profiling = prof;
                for (void* p : g->keep) (void)hipHostFree(p);
                throw;
            }
            cap = hipStreamEndCapture(st, &g->graph);
        }
        c->capturing = false;
        c->capture_host = nullptr;
        c->profiling = prof;
        if (cap != hipSuccess) {
            for (void* p : g->keep) (void)hipHostFree(p);
            throw Error{CSV_EHIP, std::string("stream capture failed: ") + hipGetErrorString(cap)};
        }
        const hipError_t e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g->graph);
            for (void* p : g->keep) (void)hipHostFree(p);
            throw Error{CSV_EHIP, std::string("graph instantiate failed: ") + hipGetErrorString(e)};
        }
        g->gen = c->gen;
        *out = g.release();
    });
}

int csv_graph_launch(csv_graph* g, void* stream) {
    return guarded([&] {
        CSV_REQUIRE(g && g->exec, CSV_EINVAL, "NULL graph");
        std::lock_guard<std::mutex> lk(g->ctx->mu);
        CSV_REQUIRE(g->gen == C(g->ctx)->gen, CSV_EINVAL,
                    "context scratch moved since capture (a larger decode on the same context "
                    "grew a buffer the graph uses); recapture");
        set_device(g->ctx);
        CSV_HIP(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    });
}

int csv_graph_destroy(csv_graph* g) {
    if (!g) return CSV_OK;
    return guarded([&] {
        (void)hipDeviceSynchronize();
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        for (void* p : g->keep) (void)hipHostFree(p);
        delete g;
    });
}

int csv_profile_enable(csv_ctx* ctx, int on) {
    return guarded([&] {
        CSV_REQUIRE(ctx, CSV_EINVAL, "ctx is NULL");
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->impl.profiling = on != 0;
    });
}

int csv_profile_query(csv_ctx* ctx, const char* name, double* total_ms, int64_t* launches) {
    return guarded([&] {
        CSV_REQUIRE(ctx && name && total_ms && launches, CSV_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(ctx->mu);
        Ctx* c = C(ctx);
        for (auto& kv : c->prof_pending) {
            auto& tot = c->prof_total[kv.first];
            for (auto& ev : kv.second) {
                CSV_HIP(hipEventSynchronize(ev.second));
                float ms = 0.f;
                CSV_HIP(hipEventElapsedTime(&ms, ev.first, ev.second));
                tot.first += ms;
                tot.second += 1;
                (void)hipEventDestroy(ev.first);
                (void)hipEventDestroy(ev.second);
            }
            kv.second.clear();
        }
        auto it = c->prof_total.find(name);
        *total_ms = it == c->prof_total.end() ? 0.0 : it->second.first;
        *launches = it == c->prof_total.end() ? 0 : it->second.second;
    });
}

int csv_profile_reset(csv_ctx* ctx) {
    return guarded([&] {
        CSV_REQUIRE(ctx, CSV_EINVAL, "ctx is NULL");
        std::lock_guard<std::mutex> lk(ctx->mu);
        Ctx* c = C(ctx);
        for (auto& kv : c->prof_pending)
            for (auto& ev : kv.second) {
                (void)hipEventSynchronize(ev.second);
                (void)hipEventDestroy(ev.first);
                (void)hipEventDestroy(ev.second);
            }
        c->prof_pending.clear();
        c->prof_total.clear();
    });
}

int csv_probe_ceilings(csv_ctx* ctx, csv_ceilings* out) {
    return guarded([&] {
        CSV_REQUIRE(ctx && out, CSV_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        int cus = 0;
        CSV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                      ctx->impl.device));
        CSV_REQUIRE(cus > 0, CSV_EHIP, "device reports no compute units");
        csv_ceilings r{};
        probe_ceilings(C(ctx), cus, &r);
        *out = r;
    });
}

int csv_phi_matrix(csv_ctx* ctx, const csv_params* p, int8_t* q_out, void* stream) {
    return guarded([&] {
        CSV_REQUIRE(ctx && q_out, CSV_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        const Shape s = resolve(p);
        hipStream_t st = static_cast<hipStream_t>(stream);
        Operator* op = get_operator(C(ctx), s, st);
        CSV_HIP(hipMemcpyAsync(q_out, op->q, (size_t)s.M * s.n, hipMemcpyDeviceToDevice, st));
    });
}

int csv_operator_matrix(csv_ctx* ctx, const csv_params* p, double* a_out, void* stream) {
    return guarded([&] {
        CSV_REQUIRE(ctx && a_out, CSV_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        const Shape s = resolve(p);
        hipStream_t st = static_cast<hipStream_t>(stream);
        CSV_REQUIRE(!(s.flags & CSV_FLAG_WHOLE_FRAME), CSV_EUNSUPPORTED,
                    "whole-frame operators have no transform basis");
        Operator* op = get_operator(C(ctx), s, st);
        CSV_HIP(hipMemcpyAsync(a_out, op->a64, (size_t)s.M * s.n * 8, hipMemcpyDeviceToDevice, st));
    });
}

int csv_step_constant(csv_ctx* ctx, const csv_params* p, double* L_out, int32_t* iters_out) {
    return guarded([&] {
        CSV_REQUIRE(ctx && L_out, CSV_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        const Shape s = resolve(p);
        Operator* op = get_operator(C(ctx), s, nullptr);
        double h[3];
        CSV_HIP(hipMemcpy(h, op->lip, sizeof(h), hipMemcpyDeviceToHost));
        *L_out = h[0];
        if (iters_out) *iters_out = (int32_t)h[2];
    });
}

int csv_key_encode(csv_ctx* ctx, int32_t width, int32_t height, int32_t qstep,
                   const uint8_t* frame, int16_t* levels, uint64_t* bits, void* stream) {
    return guarded([&] {
        CSV_REQUIRE(ctx && frame && levels, CSV_EINVAL, "NULL argument");
        csv_params p;
        csv_params_default(&p);
        p.width = width;
        p.height = height;
        p.key_qstep = qstep;
        p.gop = 1;
        const Shape s = resolve(&p);
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        hipStream_t st = static_cast<hipStream_t>(stream);
        unsigned long long* b = reinterpret_cast<unsigned long long*>(bits);
        if (b) launch_fill_u64(b, 0ull, 1, st);
        launch_key_encode(frame, s.W, s.H, s.qshift, levels, b, st);
    });
}

int csv_key_decode(csv_ctx* ctx, int32_t width, int32_t height, int32_t qstep,
                   const int16_t* levels, uint8_t* out, void* stream) {
    return guarded([&] {
        CSV_REQUIRE(ctx && levels && out, CSV_EINVAL, "NULL argument");
        csv_params p;
        csv_params_default(&p);
        p.width = width;
        p.height = height;
        p.key_qstep = qstep;
        p.gop = 1;
        const Shape s = resolve(&p);
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        launch_key_decode(levels, s.W, s.H, s.qstep, out, static_cast<hipStream_t>(stream));
    });
}

int csv_measure_frame(csv_ctx* ctx, const csv_params* p, const uint8_t* frame,
                      const uint8_t* key_decoded, int32_t* y_out, int8_t* codes, uint8_t* exps,
                      void* stream) {
    return guarded([&] {
        CSV_REQUIRE(ctx && frame && key_decoded && codes && exps, CSV_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        const Shape s = resolve(p);
        hipStream_t st = static_cast<hipStream_t>(stream);
        Ctx* c = C(ctx);
        if (s.flags & CSV_FLAG_WHOLE_FRAME) {
            // |y~| <= n 255 32 must fit y_out's int32
            CSV_REQUIRE(!y_out || (long long)s.n * 255 * 32 < (1ll << 31), CSV_EUNSUPPORTED,
                        "whole-frame measurements of this frame size exceed int32");
            long long* y = static_cast<long long*>(scratch(c, "ymeas", (size_t)s.M * 8));
            launch_whole_measure(s, frame, 1, (size_t)s.W * s.H, key_decoded, y, st);
            launch_whole_quantise(y, s.M, 1, codes, exps, y_out, st);
            return;
        }
        Operator* op = get_operator(c, s, st);
        int32_t* y = static_cast<int32_t*>(scratch(c, "ymeas", (size_t)s.nb * s.Mp * 4));
        launch_measure(s, op->q, op->q8, frame, 1, (size_t)s.W * s.H, key_decoded, y, st);
        launch_quantise(y, s.M, s.Mp, s.nb, codes, exps, y_out, st,
                        (s.flags & CSV_FLAG_NO_QUANT) != 0);
    });
}

int csv_recover_blocks(csv_ctx* ctx, const csv_params* p, int32_t n_blocks, const int8_t* codes,
                       const uint8_t* exps, float* s_out, float* lambda_out, double* obj_out,
                       void* stream) {
    return guarded([&] {
        CSV_REQUIRE(ctx && codes && exps && s_out, CSV_EINVAL, "NULL argument");
        CSV_REQUIRE(n_blocks >= 0, CSV_EINVAL, "negative block count");
        std::lock_guard<std::mutex> lk(ctx->mu);
        set_device(ctx);
        const Shape s = resolve(p);
        hipStream_t st = static_cast<hipStream_t>(stream);
        Ctx* c = C(ctx);
        CSV_REQUIRE(!(s.flags & CSV_FLAG_WHOLE_FRAME), CSV_EUNSUPPORTED,
                    "whole-frame measurements are recovered by csv_decode_gop");
        Operator* op = get_operator(c, s, st);
        recover(c, s, op, codes, exps, n_blocks, s_out, lambda_out, obj_out, st);
    });
}

}  // extern "C"
