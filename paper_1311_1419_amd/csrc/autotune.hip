// Autotuner for the fused recovery kernel: for one (n, padded M) class it
// times every compiled variant (column tiles per workgroup, prefetch ring
// depths, LDS-resident state tiles) on a synthetic operator and synthetic
// codes, keeps the fastest as the class's choice, and can persist the
// choices of every class as a small JSON file that csv_autotune_load reads.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <random>
#include <sstream>

#include "csv_tune.h"
#include "internal.h"

using namespace csv;

namespace {

std::string table_json(const std::vector<std::pair<std::string, double>>* timed, int n_t, int mp_t) {
    std::ostringstream o;
    o << "{\n  \"arch\": \"gfx950\",\n  \"classes\": [\n";
    const auto cls = fused_classes();
    for (size_t i = 0; i < cls.size(); ++i) {
        const int n = cls[i].first, mp = cls[i].second;
        const auto& v = fused_variants(n, mp);
        o << "    {\"n\": " << n << ", \"Mp\": " << mp << ", \"variant\": \""
          << v[fused_choice(n, mp)].name << "\"";
        if (timed && n == n_t && mp == mp_t) {
            o << ", \"ms\": {";
            for (size_t k = 0; k < timed->size(); ++k)
                o << (k ? ", " : "") << "\"" << (*timed)[k].first << "\": " << (*timed)[k].second;
            o << "}";
        }
        o << "}" << (i + 1 < cls.size() ? "," : "") << "\n";
    }
    o << "  ]\n}\n";
    return o.str();
}

}  // namespace

extern "C" {

int csv_autotune(csv_ctx* ctx, int32_t block, int32_t m, int32_t iters, int32_t n_blocks,
                 const char* json_path, double* ms_out, int32_t* count, int32_t* best) {
    try {
        CSV_REQUIRE(ctx && count && best, CSV_EINVAL, "NULL argument");
        CSV_REQUIRE(n_blocks > 0 && iters > 0, CSV_EINVAL, "n_blocks and iters must be positive");
        std::lock_guard<std::mutex> lk(ctx->mu);
        CSV_HIP(hipSetDevice(ctx->impl.device));
        Ctx* c = &ctx->impl;
        csv_params p;
        csv_params_default(&p);
        p.block = block;
        p.m = m;
        p.width = block * 8;
        p.height = block * 8;
        p.gop = 2;
        p.iters = iters;
        p.precision = CSV_BF16;
        p.phi_seed = 0x7475'6e65ull;   // fixed synthetic operator
        p.stream_id = 0xffffffffu;
        const Shape s = resolve(&p);
        CSV_REQUIRE(fused_class_supported(s.n, s.Mp), CSV_EUNSUPPORTED, "no fused kernel class");
        const auto& vars = fused_variants(s.n, s.Mp);
        hipStream_t st = nullptr;
        CSV_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        Operator* op = get_operator(c, s, st);
        // synthetic codes: a few large measurements over small ones, random exponents
        std::mt19937 rng(12345);
        std::vector<int8_t> codes((size_t)n_blocks * s.M);
        std::vector<uint8_t> exps(n_blocks);
        std::normal_distribution<float> g(0.f, 30.f);
        for (auto& q : codes) q = (int8_t)std::max(-127.f, std::min(127.f, std::round(g(rng))));
        for (auto& e : exps) e = (uint8_t)(rng() % 8);
        int8_t* dcodes = static_cast<int8_t*>(scratch(c, "tune_codes", codes.size()));
        uint8_t* dexps = static_cast<uint8_t*>(scratch(c, "tune_exps", exps.size()));
        float* lam = static_cast<float*>(scratch(c, "tune_lam", (size_t)n_blocks * 4));
        float* S = static_cast<float*>(scratch(c, "tune_S", (size_t)n_blocks * s.n * 4));
        CSV_HIP(hipMemcpyAsync(dcodes, codes.data(), codes.size(), hipMemcpyHostToDevice, st));
        CSV_HIP(hipMemcpyAsync(dexps, exps.data(), exps.size(), hipMemcpyHostToDevice, st));
        const float* y = prepare(c, s, op, dcodes, dexps, n_blocks, lam, "_tune", st);
        CSV_HIP(hipStreamSynchronize(st));
        // Bring the clocks up first (an idle GPU runs the first timed
        // launches slower, which biased the first variant), then time every
        // variant in two interleaved rounds and keep each one's faster round.
        {
            double spent = 0.0;
            for (int r = 0; r < 64 && spent < 150.0; ++r)
                spent += time_fused_variant(c, s, op, y, lam, S, n_blocks, fused_choice(s.n, s.Mp),
                                            1, st);
        }
        const int nv = (int)vars.size();
        std::vector<double> vms(nv, 1e300);
        for (int round = 0; round < 2; ++round)
            for (int v = 0; v < nv; ++v)
                vms[v] = std::min(vms[v], time_fused_variant(c, s, op, y, lam, S, n_blocks, v, 3, st));
        std::vector<std::pair<std::string, double>> timed;
        int bi = 0;
        double bms = 1e300;
        for (int v = 0; v < nv; ++v) {
            timed.push_back({vars[v].name, vms[v]});
            if (ms_out) ms_out[v] = vms[v];
            if (vms[v] < bms) {
                bms = vms[v];
                bi = v;
            }
        }
        CSV_HIP(hipStreamSynchronize(st));
        (void)hipStreamDestroy(st);
        set_fused_choice(s.n, s.Mp, bi);
        *count = (int32_t)vars.size();
        *best = bi;
        if (json_path && *json_path) {
            std::ofstream f(json_path);
            CSV_REQUIRE(f.good(), CSV_EINVAL, std::string("cannot write ") + json_path);
            f << table_json(&timed, s.n, s.Mp);
        }
        return CSV_OK;
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    } catch (const std::exception& e) {
        return fail(CSV_EINVAL, e.what());
    }
}

int csv_autotune_load(const char* json_path) {
    try {
        CSV_REQUIRE(json_path, CSV_EINVAL, "NULL path");
        std::ifstream f(json_path);
        CSV_REQUIRE(f.good(), CSV_ENOTFOUND, std::string("cannot read ") + json_path);
        std::string line;
        int applied = 0;
        while (std::getline(f, line)) {
            int n = 0, mp = 0;
            char name[128] = {0};
            const char* p = std::strstr(line.c_str(), "{\"n\":");
            if (!p) continue;
            if (std::sscanf(p, "{\"n\": %d, \"Mp\": %d, \"variant\": \"%127[^\"]\"", &n, &mp, name) != 3)
                continue;
            if (!fused_class_supported(n, mp)) continue;
            const auto& v = fused_variants(n, mp);
            for (int k = 0; k < (int)v.size(); ++k)
                if (std::strcmp(v[k].name, name) == 0) {
                    set_fused_choice(n, mp, k);
                    ++applied;
                }
        }
        CSV_REQUIRE(applied > 0, CSV_EINVAL, "no kernel choice recognised in the file");
        return CSV_OK;
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    }
}

int csv_autotune_choice(int32_t block, int32_t m, char* name, size_t name_len, int32_t* index,
                        int32_t* count) {
    try {
        csv_params p;
        csv_params_default(&p);
        p.block = block;
        p.m = m;
        const Shape s = resolve(&p);
        const auto& v = fused_variants(s.n, s.Mp);
        const int k = fused_choice(s.n, s.Mp);
        if (index) *index = k;
        if (count) *count = (int32_t)v.size();
        if (name && name_len) {
            std::strncpy(name, v[k].name, name_len - 1);
            name[name_len - 1] = 0;
        }
        return CSV_OK;
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    }
}

int csv_autotune_set(int32_t block, int32_t m, int32_t index) {
    try {
        csv_params p;
        csv_params_default(&p);
        p.block = block;
        p.m = m;
        const Shape s = resolve(&p);
        set_fused_choice(s.n, s.Mp, index);
        return CSV_OK;
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    }
}

}  // extern "C"
