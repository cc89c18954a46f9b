// Internal declarations of the HIP library behind include/csv.h.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "csv.h"

namespace csv {

// ---------------------------------------------------------------- errors
struct Error {
    int code;
    std::string msg;
};
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define CSV_HIP(expr)                                                        \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess)                                                \
            throw ::csv::Error{CSV_EHIP, std::string(#expr) + ": " +         \
                                             hipGetErrorString(e_)};         \
    } while (0)

#define CSV_REQUIRE(cond, code, msg)                                         \
    do {                                                                     \
        if (!(cond)) throw ::csv::Error{(code), (msg)};                      \
    } while (0)

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline int round_up(int a, int b) { return ceil_div(a, b) * b; }

// Resolved, validated parameter set.
struct Shape {
    int W, H, G, B, n, M, Mp, nbx, nby, nb;   // nb: blocks per frame
    int qstep, qshift, T;
    float lambda_frac;
    int precision, flags;
    uint64_t seed;
    uint32_t sid;
};
Shape resolve(const csv_params* p);

// Per-stream operator state, resident in HBM while the context lives.
struct Operator {
    int B = 0, n = 0, M = 0, Mp = 0;
    bool whole = false;           // whole-frame operator: q, qt and lip only
    int8_t* qt = nullptr;         // whole frame: n x Mp, Q transposed
    uint64_t seed = 0;
    uint32_t sid = 0;
    double s_phi = 0;
    int8_t* q = nullptr;          // Mp x n, rows >= M zero
    uint8_t* q8 = nullptr;        // Mp x n, Q as OCP E4M3 bytes (FP8 measurement form)
    double* a64 = nullptr;        // Mp x n, A = s_phi Q Psi (final FP64 check)
    float* a32 = nullptr;         // Mp x n
    float* phi32 = nullptr;       // Mp x n, s_phi Q
    uint8_t* qb_fwd = nullptr;    // Q + 64, forward fragment order (int8-Q fused kernel)
    uint8_t* qb_adj = nullptr;    // Q + 64, adjoint fragment order
    uint16_t* frag_fwd = nullptr; // bf16 A in forward-product fragment order
    uint16_t* frag_adj = nullptr; // bf16 A in adjoint-product fragment order
    uint16_t* phi_frag_fwd = nullptr;   // bf16 Phi, forward fragment order (TV)
    uint16_t* phi_frag_adj = nullptr;   // bf16 Phi, adjoint fragment order (TV)
    double* lip = nullptr;        // device: [0] L_used, [1] Rayleigh quotient, [2] iterations
    float* dct = nullptr;         // B x B orthonormal DCT-II, C[k][i]
    double* dct64 = nullptr;      // same in FP64
    size_t bytes = 0;
};

// Scratch buffers owned by a context, grown on demand.
struct Scratch {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Per-stream operators, shareable between contexts (the server's batch
// slots share one cache; each csv_ctx owns its own).
struct OpCache {
    std::mutex mu;
    // (seed, stream, n, M, whole frame)
    std::map<std::tuple<uint64_t, uint32_t, int, int, bool>, std::unique_ptr<Operator>> ops;
};

struct Ctx {
    int device = 0;
    std::shared_ptr<OpCache> cache = std::make_shared<OpCache>();
    size_t budget = 0;
    size_t used = 0;
    void* stage_host = nullptr;      // pinned staging for tile descriptors
    size_t stage_bytes = 0;
    hipEvent_t stage_done = nullptr;
    bool profiling = false;
    std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> prof_pending;
    std::map<std::string, std::pair<double, long long>> prof_total;
    std::map<std::string, Scratch> scratch;
    std::map<int, std::pair<float*, int>> beta_tables;   // key: T*2 + ista
    int gen = 0;   // bumps whenever a scratch buffer moves
    // Stream capture: tile tables go to pinned buffers owned by the graph
    // (capture_host) instead of the reusable staging buffer, and no host
    // synchronisation or allocation may happen.
    bool capturing = false;
    void* capture_host = nullptr;     // pinned tile table owned by the graph
    size_t capture_bytes = 0;
    size_t last_table_bytes = 0;      // size of the latest tile table upload
    // Auxiliary streams: per-GOP kernels of a batch decode (key frames,
    // lambda, FP64 check, synthesis) are spread over them, forked from and
    // joined back into the caller's stream with events.
    static constexpr int kAux = 3;
    hipStream_t aux[kAux] = {};
    hipEvent_t aux_done[kAux] = {};
    hipEvent_t fork_ev = nullptr;
};

// Records a pair of events around a named kernel range when profiling is on.
class ProfScope {
  public:
    ProfScope(Ctx* c, const char* name, hipStream_t st);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

  private:
    Ctx* c_;
    const char* name_;
    hipStream_t st_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

// allocation inside the context budget
void* ctx_alloc(Ctx* c, size_t bytes);
void ctx_free(Ctx* c, void* p, size_t bytes);
void* scratch(Ctx* c, const std::string& name, size_t bytes);
Operator* get_operator(Ctx* c, const Shape& s, hipStream_t st);
// Build the operators of every shape not yet cached, with one batched power
// iteration for all of them (the setup of many new streams at once).
void prepare_operators(Ctx* c, const Shape* shapes, int count, hipStream_t st);
void free_operators(Ctx* c);   // when c holds the last reference to its cache
void release_ctx(Ctx* c);      // free everything c allocated
// Decode `count` GOPs (key frames, recovery of every CS block in one pass,
// synthesis); the body of csv_decode_gop / csv_decode_batch.
double time_fused_variant(Ctx* c, const Shape& s, Operator* op, const float* y, const float* lam,
                          float* S, int nblk, int variant, int reps, hipStream_t st);
// lambda's adjoint product goes to scratch buffer `g0name`
const float* prepare(Ctx* c, const Shape& s, Operator* op, const int8_t* codes,
                     const uint8_t* exps, int nblk, float* lam, const std::string& tag,
                     hipStream_t st, const std::string& g0name = "g0");
// Encode `count` GOPs; the body of csv_encode_gop / csv_encode_batch.
void encode_gops(Ctx* c, int count, const Shape* shapes, const uint8_t* const* frames,
                 const csv_gop_stream* out, hipStream_t st);
void decode_gops(Ctx* c, int count, const Shape* shapes, const csv_gop_stream* in,
                 uint8_t* const* frames_out, float* const* cs_float_out, double* const* obj_out,
                 hipStream_t st);
const float* beta_table(Ctx* c, int T, bool ista, hipStream_t st);
// (t_k / t_{k+1}, (t_k - 1) / t_{k+1}) for k = 1..T, interleaved (monotone FISTA)
const float* mfista_table(Ctx* c, int T, hipStream_t st);

// ------------------------------------------------------------- kernels
// encode side (k_encode.hip)
void launch_phi_q(int8_t* q, int M, int Mp, int n, uint64_t k0, uint64_t k1, hipStream_t st);
void launch_key_encode(const uint8_t* frame, int W, int H, int qshift, int16_t* levels,
                       unsigned long long* bits, hipStream_t st);
void launch_key_decode(const int16_t* levels, int W, int H, int qstep, uint8_t* out, hipStream_t st);
// exact BF16-MFMA product, or the INT8 / FP8 form selected by s.flags
void launch_measure(const Shape& s, const int8_t* q, const uint8_t* q8, const uint8_t* frames,
                    int n_frames, size_t frame_stride, const uint8_t* key, int32_t* y_scratch,
                    hipStream_t st);
// raw: store y~ as int32 at codes, exponents 0 (CSV_FLAG_NO_QUANT)
void launch_quantise(const int32_t* y, int M, int Mp, int total, int8_t* codes, uint8_t* exps,
                     int32_t* y_out, hipStream_t st, bool raw = false);
void launch_q_e4m3(const int8_t* q, uint8_t* q8, size_t count, hipStream_t st);
void launch_fill_u64(unsigned long long* p, unsigned long long v, int count, hipStream_t st);

// decode side (k_decode.hip)
void launch_operator_setup(Operator* op, hipStream_t st);
// The exact Gram matrix QQ^T is stored row-major with rows padded to
// gram_ld(M) int32 (zero beyond column M), so rows start 16-byte aligned.
__host__ __device__ inline int gram_ld(int M) { return (M + 3) & ~3; }
// Scratch a power iteration needs beside G (its many-workgroup form's row
// slices, iterates and state; 0 where the one-workgroup forms run)
size_t power_work_bytes(int M);
void launch_power_iteration(Operator* op, int* gram, void* work,
                            hipStream_t st);   // gram: M x gram_ld(M) scratch
// The same for many operators: each one's exact Gram matrix (launch_gram),
// then their power iterations side by side, one workgroup per operator,
// kPowBatch operators per launch.
constexpr int kPowBatch = 64;
struct PowJob {
    const int* gram;
    int M, S;
    double s_phi;
    double* lip;
};
struct PowBatch {
    PowJob j[kPowBatch];
};
void launch_gram(Operator* op, int* gram, hipStream_t st);
void launch_power_batch(Operator* const* ops, int* const* grams, int count, void* work,
                        hipStream_t st);
// raw: codes hold int32 y~ and exps are ignored (CSV_FLAG_NO_QUANT)
void launch_dequant(const int8_t* codes, const uint8_t* exps, int nblk, int M, int Mp,
                    double s_phi, float* y, hipStream_t st, bool raw = false);
void launch_row_absmax(const float* X, int R, int N, int ld, float scale, float* out, hipStream_t st);
void launch_fill_f32(float* p, float v, size_t count, hipStream_t st);
void launch_copy_f32(float* dst, const float* src, size_t count, hipStream_t st);
void launch_synth(const float* s, const float* dct, const uint8_t* key, int W, int H, int B,
                  int nbx, int nb, int n_frames, uint8_t* out_u8, float* out_f32, hipStream_t st);
// FP64 final check of the DCT-l1 recovery for up to kF64Batch GOPs of one
// (n, M, Mp) shape in one launch (grid.y = GOP).
struct F64Job {
    const double* a64;      // Mp x n operator (FP64)
    const float* s;         // nblk x n coefficients
    const int8_t* codes;    // nblk x M
    const uint8_t* exps;    // nblk
    const float* lam;       // nblk
    double* obj;            // nblk x 2
    double s_phi;
    int nblk;
    int raw = 0;            // codes hold int32 y~ (CSV_FLAG_NO_QUANT)
};
constexpr int kF64Batch = 16;
struct F64Batch {
    F64Job j[kF64Batch];
};
void launch_final64_batch(const F64Batch& bt, int ngop, int M, int Mp, int n, hipStream_t st);
void launch_final64(const double* a64, const float* s, const int8_t* codes, const uint8_t* exps,
                    const float* lam, int nblk, int M, int Mp, int n, double s_phi, double* obj,
                    hipStream_t st, bool raw = false);

// set-up of csv_measure_frame_noalloc's device array on the current device
// (noalloc.hip), once per device
void noalloc_setup(int dev);

// device ceilings (k_probe.hip); synchronous
void probe_ceilings(Ctx* c, int cus, csv_ceilings* out);

// whole-frame measurement (k_whole.hip): y (n_frames x M, int64)
void launch_whole_measure(const Shape& s, const uint8_t* frames, int n_frames, size_t frame_stride,
                          const uint8_t* key, long long* y, hipStream_t st);
void launch_whole_quantise(const long long* y, int M, int n_frames, int8_t* codes, uint8_t* exps,
                           int32_t* y32, hipStream_t st);
// whole-frame recovery: products with the resident int8 Q, output, FP64 check
// Plain FP32 recovery of a batch of up to kF32Batch GOPs of one shape
// (k_fp32_mfma.hip): per GOP its operator (M_p x n FP32: A for l1, Phi for
// TV), its dequantised y^ (nblk x M_p), lambda, step constant, and the
// iterates s, v, gradient G (nblk x n) and residual R (nblk x M_p).
constexpr int kF32Batch = 16;
struct F32Job {
    const float* op;
    const float* y;      // forward: R = V A^T - y^, or V A^T itself when NULL
    const float* lam;
    const double* lip;
    float* S;
    float* V;
    float* G;
    float* R;
    int nblk;
    // monotone FISTA only: z_k (nblk x n), A z_k and A s_k (nblk x Mp) and
    // F(s_k) per block (FP64)
    float* Z = nullptr;
    float* AZ = nullptr;
    float* AS = nullptr;
    double* FS = nullptr;
};
struct F32Batch {
    F32Job j[kF32Batch];
};
// R = V A^T - y^ (rows m < M; zero for M <= m < M_p), on FP32 MFMA
void launch_f32_forward(const F32Batch& bt, int ngop, int n, int M, int Mp, hipStream_t st);
// G = R A, on FP32 MFMA
void launch_f32_adjoint(const F32Batch& bt, int ngop, int n, int Mp, hipStream_t st);
// G = R A with the FISTA step of iteration k applied to each output in
// place of storing it: u = V - G / L, S = soft(u, lam / L),
// V = S + beta_k (S - S_prev); G is not written
void launch_f32_adjoint_prox(const F32Batch& bt, int ngop, int n, int Mp, const float* beta,
                             int k, hipStream_t st);
// Monotone FISTA (CSV_FLAG_MONOTONE), with S, V, Z, AZ, AS, FS of each job:
//   init:   S = V = 0, A s_0 = 0, R = -y^, F(s_0) = 1/2 ||y^||^2;
//   zstep:  G = R A and z_k = soft(V - G / L, lam / L) into Z (G not stored);
//   select: per block F(z_k) = 1/2 ||A z_k - y^||^2 + lam ||z_k||_1 (FP64
//           sums in a fixed order), s_k = z_k if F(z_k) <= F(s_{k-1}) else
//           s_{k-1}, v_{k+1} = s_k + c1 (z_k - s_k) + c2 (s_k - s_{k-1}), the
//           same combination for A s_k and A v_{k+1}, and R = A v_{k+1} - y^;
//           coef[k] = (c1, c2) = (t_k / t_{k+1}, (t_k - 1) / t_{k+1}).
// The forward product A z_k is launch_f32_forward on a batch whose V is Z,
// R is AZ and y is NULL.
void launch_mfista_init(const F32Batch& bt, int ngop, int n, int M, int Mp, hipStream_t st);
void launch_f32_adjoint_zstep(const F32Batch& bt, int ngop, int n, int Mp, hipStream_t st);
void launch_mfista_select(const F32Batch& bt, int ngop, int n, int M, int Mp, const float* coef,
                          int k, hipStream_t st);

// A batch of up to kWholeBatch GOPs of one shape, each with its own Q
// (passed by value as a kernel argument); x, y, r are [GOP][F][.] arrays.
constexpr int kWholeBatch = 16;
struct WholeQ {
    const int8_t* q[kWholeBatch];
};
struct WholeLip {
    const double* lip[kWholeBatch];
};
// TV state of a batch ([GOP][F][n] arrays, lam [GOP][F], lip [GOP]); all
// null for a plain product
struct WholeTv {
    float* x;
    float *nuh, *nuv, *wh, *wv, *ph, *pv;
    const float* lam;
    const float* alpha;   // per image: 1 / (L_g + 8 beta)
};
int whole_fwd_parts(int n);
// forward: r = s_Phi Q x - y^ through whole_fwd_parts(n) partials (part:
// that many x GOPs x F x M floats), with the TV dual step when tv.nuh is set
void launch_whole_fwd(const WholeQ& qs, int ngop, const float* x, int F, int H, int W, int M,
                      float s_phi, const float* y, float* part, float* r, const WholeTv& tv,
                      hipStream_t st);
// adjoint from Q^T (n x Mp): gout = s_Phi Q^T r, or with tv.nuh set the TV
// primal step x <- x - alpha (s_Phi Q^T r + D^T P)
void launch_whole_adj(const WholeQ& qts, int ngop, const float* r, int F, int H, int W, int M,
                      int Mp, float s_phi, float* gout, const WholeTv& tv, hipStream_t st);
void launch_transpose_q(const int8_t* q, int Mp, int n, int8_t* qt, hipStream_t st);
// alpha[b] = 1 / (L_g + 8 beta(lam[b])) for image b = g F + f of a batch
void launch_whole_alpha(const WholeLip& ls, const float* lam, int F, int ngop, float* alpha,
                        hipStream_t st);
void launch_whole_place(const float* x, const uint8_t* key, int F, int n, uint8_t* out,
                        float* out_f32, hipStream_t st);
void launch_whole_objective(const int8_t* q, const float* x, int F, int H, int W, int M,
                            double s_phi, const int8_t* codes, const uint8_t* exps,
                            const float* lam, double* rr, double* yy, double* obj,
                            hipStream_t st);

// total-variation recovery (k_tv.hip)
void launch_tv_dual(const float* x, float* nuh, float* nuv, float* wh, float* wv, float* ph,
                    float* pv, const float* lam, int nblk, int BH, int BW, hipStream_t st);
void launch_tv_primal(float* x, const float* g, const float* ph, const float* pv,
                      const float* alpha, int nblk, int BH, int BW, hipStream_t st);
// alpha[b] = 1 / (L + 8 beta(lam[b])) for count images of one operator (lip: its L)
void launch_tv_alpha(const double* lip, const float* lam, int count, float* alpha,
                     hipStream_t st);
void launch_tv_final64(const int8_t* q, const float* x, const int8_t* codes, const uint8_t* exps,
                       const float* lam, int nblk, int M, int B, double s_phi, double* obj,
                       hipStream_t st);

// fused BF16 recovery (k_fista_bf16.hip)
struct FusedTile {
    const uint16_t* frag_fwd;
    const uint16_t* frag_adj;
    const uint8_t* qb_fwd;   // Q + 64 in forward fragment order (k_fista_q8.hip)
    const uint8_t* qb_adj;   // Q + 64 in adjoint fragment order
    const float* dct;        // B x B DCT table
    float s_phi;
    const double* lip;
    const float* y;      // nblk x Mp
    const float* lam;    // nblk
    float* s;            // nblk x n
    const float* beta;   // T momentum factors
    int nblk;            // blocks in this tile (<= tile width)
    int T;
    int n, Mp;
};
void launch_bf16_frag_layout(Operator* op, hipStream_t st);
void launch_q8_frag_layout(Operator* op, hipStream_t st);
void launch_fista_q8_m256(const FusedTile* tiles, const int* qoff, const int* queue,
                          int* counters, int grid, hipStream_t st);
struct FusedVariant {
    const char* name;
    int ct;    // column tiles of 32 blocks per workgroup
    int occ;   // workgroups resident per CU
    void (*launch)(const FusedTile*, const int*, const int*, int*, int, hipStream_t);
};
bool fused_class_supported(int n, int Mp);
const std::vector<FusedVariant>& fused_variants(int n, int Mp);
int fused_choice(int n, int Mp);
void set_fused_choice(int n, int Mp, int idx);
std::vector<std::pair<int, int>> fused_classes();
int fused_tile_blocks(int n, int Mp);   // blocks per tile of the chosen variant
// one persistent launch over the `count` tiles of one (n, Mp) class;
// qoff[0..8] delimit eight per-XCD queues of tile indices, counters[8] start
// at zero; variant < 0 selects the class's current choice.  The grid is
// min(count, CUs x the variant's workgroups per CU).
void launch_fista_bf16_class(int n, int Mp, const FusedTile* tiles, const int* qoff,
                             const int* queue, int* counters, int count, hipStream_t st,
                             int variant = -1);
// Raise kernel FN's dynamic LDS limit to `bytes` on the current device, once
// per device (the attribute is per device; concurrent first calls may both
// set it, which is harmless).
template <auto FN>
inline void ensure_lds_limit(size_t bytes) {
    static std::atomic<uint64_t> done{0};   // one bit per device ordinal < 64
    int dev = 0;
    CSV_HIP(hipGetDevice(&dev));
    const uint64_t bit = 1ull << (dev & 63);
    if (done.load(std::memory_order_acquire) & bit) return;
    CSV_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(FN),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    done.fetch_or(bit, std::memory_order_release);
}

int device_cus();
// fused BF16 TV recovery (k_tv_bf16.hip): 16 x 16 blocks, tiles of 32
bool tv_class_supported(int n, int Mp);
void launch_tv_bf16_class(int n, int Mp, const FusedTile* tiles, const int* qoff,
                          const int* queue, int* counters, int count, int cus, hipStream_t st);

}  // namespace csv

// The opaque handle of csv.h.
struct csv_ctx {
    csv::Ctx impl;
    std::mutex mu;
};
