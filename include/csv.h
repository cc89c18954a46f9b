/*
 * csv.h - C ABI of the MI355X (gfx950) multiple-residual compressive-sensing
 * video coder.
 *
 * Method (Yu, Qiao, Luo, Yang, "Increasing compression ratio of low
 * complexity compressive sensing video encoder with application-aware
 * configurable mechanism"):
 *   - a GOP is one key frame plus G-1 CS frames (Section 3, Table I);
 *   - the key frame is intra coded; every CS frame subtracts the *decoded*
 *     key frame (Section 3.2, eqs. (2)-(3));
 *   - each CS-frame residual is measured with a random matrix (Section 3.1),
 *     here per B x B block with one seeded matrix per stream;
 *   - the decoder recovers the residual by sparse recovery (eq. (1)), here a
 *     LASSO in the per-block 2-D DCT basis solved by FISTA, and adds the
 *     decoded key frame back (eq. (4)).
 *
 * Conventions for every entry point:
 *   - return value: CSV_OK (0) or a negative CSV_E* code; on error
 *     csv_last_error() returns a message (thread-local, valid until the next
 *     call on the same thread).  No C++ exception crosses this boundary.
 *   - "device" pointers are HIP device memory on the context's device,
 *     owned by the caller; the library never frees caller memory.
 *   - work is enqueued on the given stream (a hipStream_t, NULL = the
 *     default stream) and is complete once that stream synchronises;
 *     entry points documented as synchronous wait for it themselves.
 *   - a context serves one host thread at a time; its scratch buffers are
 *     reused by every call, so calls that may overlap on the device must be
 *     issued on one stream (or on different contexts).
 *   - frames are uint8 luma, H rows x W columns, row-major.
 *   - N_b = ceil(H/B) * ceil(W/B) blocks per frame, numbered row-major;
 *     a block's pixels are vectorised row-major (n = B*B); residuals are
 *     zero-padded to whole blocks.
 */
#ifndef CSV_H
#define CSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- status */
enum {
    CSV_OK = 0,
    CSV_EINVAL = -1,        /* invalid argument or parameter set */
    CSV_EUNSUPPORTED = -2,  /* valid but not supported by this build */
    CSV_ENOMEM = -3,        /* memory budget or device allocation exhausted */
    CSV_EAGAIN = -4,        /* server queue full: retry later */
    CSV_EHIP = -5,          /* HIP runtime error */
    CSV_ENOTFOUND = -6,     /* unknown ticket or stream id */
    CSV_ECANCELED = -7      /* request was cancelled */
};

/* ------------------------------------------------- precision and flags */
enum {
    CSV_FP32 = 0,   /* plain FP32 path: separate GEMM / residual / threshold passes */
    CSV_BF16 = 1    /* fused path: BF16 MFMA products, FP32 accumulation and iterates */
};

enum {
    CSV_FLAG_ISTA = 1,                 /* no momentum (t_k = 1): proximal gradient */
    CSV_FLAG_LAMBDA_PIXEL_DOMAIN = 2,  /* lambda = frac*||Phi^T y||_inf instead of ||(Phi Psi)^T y||_inf */
    /* Encoder measurement forms (a low-complexity encoder, Sections 1 and 3;
     * at most one of the two):
     *   INT8: y~ = 16 Q h + Q l with r = 16 h + l, l in [0, 15], on int8
     *         MFMA with int32 accumulation; identical to the exact y~ = Q r;
     *   FP8:  y~ = e4m3(Q) e4m3(r), OCP E4M3 operands (round to nearest
     *         even) on FP8 MFMA; every E4M3 value of these integers is an
     *         integer and the FP32 sums stay below 2^24, so y~ is that exact
     *         integer sum, a few percent away from Q r.
     * The decoder ignores these flags. */
    CSV_FLAG_MEASURE_INT8 = 4,
    CSV_FLAG_MEASURE_FP8 = 8,
    /* Decoder: total-variation recovery (the paper's TVAL3-style solver,
     * Section 4) instead of l1 in the DCT basis: per block, in the pixel
     * domain, min lam TV(x) + 1/2 ||Phi x - y^||^2 with isotropic TV over
     * forward differences inside the block, by the linearised alternating-
     * direction iteration (w = shrink(D x + nu/beta, lam/beta); one gradient
     * step on x with step 1/(L + 8 beta); nu += beta (D x - w)); beta = 0.03
     * lam; lam = lambda_frac ||Phi^T y^||_inf.  CSV_FP32: any block size;
     * CSV_BF16 (fused, BF16 products, FP32 iterates): 16 x 16 blocks with
     * M up to 128, CSV_EUNSUPPORTED otherwise.  obj_out then holds the TV
     * objective. */
    CSV_FLAG_TV = 16,
    /* Encoder: whole-frame measurement, eq. (1) read literally: each CS
     * frame's residual is one vector of n = W H pixels (block is ignored,
     * N_b = 1, M up to W H, m = 0 takes M = floor(rho W H + 0.5)), measured
     * by the M x (W H) matrix of the same counter generator, regenerated
     * inside the kernel and never stored, in exact 64-bit integer sums, and
     * quantised as one block per frame.  GOPs of at most 32 frames; exact
     * integer form only.  Decoder: each CS frame is recovered as one H x W
     * image by the TV solver above (needs CSV_FLAG_TV and CSV_FP32;
     * CSV_EUNSUPPORTED otherwise), with Q (M x W H int8)
     * resident on the device and L from the FP64 power iteration on Q Q^T
     * (M <= 16384); obj_out holds one (objective, relative residual) pair per
     * CS frame.  csv_recover_blocks and csv_operator_matrix refuse it. */
    CSV_FLAG_WHOLE_FRAME = 32,
    /* Decoder: monotone FISTA (MFISTA, Beck and Teboulle 2009, the variant
     * whose objective never increases; the check of a decreasing objective
     * of eq. (1) read as a LASSO): each iteration takes the prox step z_k from
     * v_k, keeps s_k = z_k if F(z_k) <= F(s_{k-1}) and s_k = s_{k-1}
     * otherwise (per block), and extrapolates v_{k+1} = s_k + (t_k/t_{k+1})
     * (z_k - s_k) + ((t_k - 1)/t_{k+1}) (s_k - s_{k-1}).  Still two products
     * per iteration: A z_k is computed, A s_k and A v_{k+1} are carried as
     * the same combinations.  DCT-l1 recovery on the plain FP32 path only
     * (CSV_EUNSUPPORTED with CSV_BF16); CSV_EINVAL with CSV_FLAG_ISTA or
     * CSV_FLAG_TV. */
    CSV_FLAG_MONOTONE = 64,
    /* Test hook for the closed loop of eqs. (2)-(4): the encoder skips the
     * 8-bit quantiser and stores the exact integer measurements y~ = Q r as
     * int32 in `codes` ((G-1)*N_b*M int32, 4-byte aligned; csv_encoded_size
     * reports their bytes and 32 M bits per block); exps are written as 0.
     * The decoder recovers from y^ = s_Phi y~.  Block DCT-l1 recovery only
     * (CSV_EUNSUPPORTED with CSV_FLAG_TV or CSV_FLAG_WHOLE_FRAME). */
    CSV_FLAG_NO_QUANT = 128
};

/* ------------------------------------------------------------ params */
/* One stream's coding parameters (Section 2: GOP size and measurement
 * matrix size are configurable).  Validation rules (CSV_EINVAL otherwise):
 * width, height > 0 and multiples of 8; block in {16, 32}; gop >= 1
 * (gop = 1 is a key-frame-only GOP); 1 <= m <= block*block (m = 0 means
 * m = floor(rho*n + 0.5)); key_qstep a power of two in [1, 256];
 * iters >= 1; lambda_frac >= 0; precision CSV_FP32 or CSV_BF16.
 * n = block*block <= 2048 keeps the integer measurement exact in FP32. */
typedef struct {
    int32_t width;
    int32_t height;
    int32_t gop;          /* frames per GOP, key frame included */
    int32_t block;        /* B: 16 or 32 */
    int32_t m;            /* measurements per block (0: from rho) */
    float rho;            /* M/n when m == 0 */
    uint64_t phi_seed;    /* measurement-matrix key word 0 */
    uint32_t stream_id;   /* measurement-matrix key word 1 */
    int32_t key_qstep;    /* key-frame quantiser step (16) */
    int32_t iters;        /* FISTA iterations T */
    float lambda_frac;    /* lambda = lambda_frac * ||A^T y||_inf (0.01) */
    int32_t precision;    /* CSV_FP32 | CSV_BF16 */
    int32_t flags;        /* CSV_FLAG_* */
} csv_params;

/* Encoded GOP (Fig. 3: key-frame stream plus CS measurements).  All
 * pointers are device memory owned by the caller, sized by
 * csv_encoded_size().
 *   key_levels: H*W int16 quantised integer-DCT levels, each 8x8 block of
 *               levels stored at its block's position (row = vertical
 *               frequency);
 *   codes:      (G-1)*N_b*M int8, frame-major, block-major, M contiguous;
 *               values in [-127, 127];
 *   exps:       (G-1)*N_b uint8 per-block power-of-two exponents;
 *   bits:       2 uint64 written by the encoder: [0] key-frame bits
 *               (Exp-Golomb count), [1] CS bits = (G-1)*N_b*(8M+8);
 *               ignored (may be NULL) on decode. */
typedef struct {
    int16_t* key_levels;
    int8_t* codes;
    uint8_t* exps;
    uint64_t* bits;
} csv_gop_stream;

typedef struct csv_ctx csv_ctx;

/* ----------------------------------------------------------- context */
/* Create a context on HIP device `device`.  mem_budget bounds the bytes the
 * context itself allocates (stream caches, scratch); 0 = no bound. */
int csv_create(csv_ctx** out, int device, size_t mem_budget);
int csv_destroy(csv_ctx* ctx);
const char* csv_last_error(void);
const char* csv_version(void);
/* Bytes currently held by the context. */
int csv_ctx_bytes(const csv_ctx* ctx, size_t* bytes);

/* ------------------------------------------------- sizes and arithmetic */
/* Fill p with the defaults (key_qstep 16, iters 300, lambda_frac 0.01,
 * block 16, gop 4, rho 0.25, CSV_BF16). */
int csv_params_default(csv_params* p);
/* Validate p and report the measurement count M and blocks per frame. */
int csv_resolve(const csv_params* p, int32_t* m, int32_t* blocks_per_frame);
/* Element counts of the encoded GOP buffers and the CS bit count. */
int csv_encoded_size(const csv_params* p, size_t* key_elems, size_t* code_bytes,
                     size_t* exp_bytes, uint64_t* bits_cs);
/* Compression ratios from bit counts (Table I): raw GOP bits 8*G*H*W over
 * key bits plus CS bits; per-part ratios as raw bits of that part over its
 * coded bits.  Any output may be NULL. */
int csv_compression_ratio(const csv_params* p, uint64_t bits_key, uint64_t bits_cs,
                          double* total, double* key, double* cs);

/* -------------------------------------------------------- hot path */
/* Encode one GOP (Section 3.1, Fig. 3).  frames: device, G*H*W uint8.
 * Frame 0 is the key frame; frames 1..G-1 are measured against the decoded
 * key frame.  Asynchronous on `stream`. */
int csv_encode_gop(csv_ctx* ctx, const csv_params* p, const uint8_t* frames,
                   const csv_gop_stream* out, void* stream);

/* Encode `count` GOPs, possibly of different streams and sizes, with the
 * same results as `count` csv_encode_gop calls.  params[i], frames[i] and
 * out[i] describe GOP i (host arrays of `count` entries; frames[i] and the
 * buffers of out[i] are device memory as for csv_encode_gop).  The GOPs'
 * kernels overlap on the device.  Asynchronous on `stream`. */
int csv_encode_batch(csv_ctx* ctx, int32_t count, const csv_params* params,
                     const uint8_t* const* frames, const csv_gop_stream* out, void* stream);

/* Decode one GOP (Section 3.2, Fig. 4, eqs. (1) and (4)).
 *   frames_out:   device, G*H*W uint8; frame 0 = decoded key frame;
 *   cs_float_out: device, (G-1)*H*W float (decoded key + recovered
 *                 residual before rounding), or NULL;
 *   obj_out:      device, (G-1)*N_b*2 double, per block the FP64 LASSO
 *                 objective 1/2||A s - y||^2 + lam||s||_1 and the relative
 *                 residual ||A s - y|| / ||y||, or NULL.
 * Asynchronous on `stream`. */
int csv_decode_gop(csv_ctx* ctx, const csv_params* p, const csv_gop_stream* in,
                   uint8_t* frames_out, float* cs_float_out, double* obj_out,
                   void* stream);

/* Decode `count` GOPs, possibly of different streams, sizes, M and block
 * sizes, in one pass: every recovery block of every GOP goes through one
 * launch of the fused recovery kernel (precision CSV_BF16) or one FISTA
 * pass of the plain path (all entries CSV_FP32); mixing precisions in one
 * batch is CSV_EINVAL.  Arrays have `count` entries; cs_float_out and
 * obj_out may be NULL (or hold NULL entries). */
int csv_decode_batch(csv_ctx* ctx, int32_t count, const csv_params* params,
                     const csv_gop_stream* in, uint8_t* const* frames_out,
                     float* const* cs_float_out, double* const* obj_out,
                     void* stream);

/* ------------------------------------------ single steps of the path */
/* Measurement matrix Q (Section 3.1 "random matrix"; Philox4x64-10 of
 * Salmon et al., SC'11): q_out device int8 M x n row-major, entries
 * popcount(word) - 32 in [-32, 32]; Phi = Q / (4 sqrt(M)). */
int csv_phi_matrix(csv_ctx* ctx, const csv_params* p, int8_t* q_out, void* stream);

/* Operator A = Phi Psi (FP64, M x n row-major, device) with Psi the
 * orthonormal 2-D DCT-II synthesis of a B x B block. */
int csv_operator_matrix(csv_ctx* ctx, const csv_params* p, double* a_out, void* stream);

/* Step constant L = 1.001 * ||Phi||_2^2 from the FP64 power iteration on
 * the integer Gram matrix Q Q^T.  Synchronous; writes the host double
 * *L_out and the iteration count (may be NULL). */
int csv_step_constant(csv_ctx* ctx, const csv_params* p, double* L_out, int32_t* iters_out);

/* Key-frame stand-in codec (integer 8x8 DCT, uniform power-of-two step,
 * Exp-Golomb bit count).  frame/out: device H*W uint8; levels: device
 * H*W int16; bits: device uint64 (one value), may be NULL. */
int csv_key_encode(csv_ctx* ctx, int32_t width, int32_t height, int32_t qstep,
                   const uint8_t* frame, int16_t* levels, uint64_t* bits, void* stream);
int csv_key_decode(csv_ctx* ctx, int32_t width, int32_t height, int32_t qstep,
                   const int16_t* levels, uint8_t* out, void* stream);

/* Measure one CS frame against a decoded key frame (Section 3.2 eq. (3)
 * residual; y = Q r per block, exact integers): y_out device int32
 * N_b x M (may be NULL), codes device int8 N_b x M, exps device uint8 N_b. */
int csv_measure_frame(csv_ctx* ctx, const csv_params* p, const uint8_t* frame,
                      const uint8_t* key_decoded, int32_t* y_out, int8_t* codes,
                      uint8_t* exps, void* stream);

/* csv_measure_frame without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and results as csv_measure_frame,
 * minus the context, plus the measurement matrix the caller holds:
 *   q: device int8 M x n row-major, as written by csv_phi_matrix for p.
 * Runs on the calling thread's current HIP device.  Its working memory is
 * a file-scope device array of 16 MiB per device (padded Q, Q as E4M3 for
 * CSV_FLAG_MEASURE_FP8, and the N_b x M_p int32 measurements; M_p = M
 * rounded up to 32), held by each device the library runs on until the
 * process ends; every byte a call reads there is first written by that
 * call.  Frames needing more (about 3.5 M block-measurements, e.g. beyond
 * 1920x1088 at M/n = 0.25) return CSV_EINVAL before any GPU work, as do the
 * other validation errors; whole-frame measurement returns
 * CSV_EUNSUPPORTED.  Every call on one device shares that array: calls that
 * overlap on one device (different streams, or different host threads)
 * race and must be serialised by the caller. */
int csv_measure_frame_noalloc(const csv_params* p, const int8_t* q, const uint8_t* frame,
                              const uint8_t* key_decoded, int32_t* y_out, int8_t* codes,
                              uint8_t* exps, void* stream);

/* Recover n_blocks residual blocks of one stream from their codes
 * (eq. (1) as a LASSO, FISTA): s_out device float n_blocks x n DCT
 * coefficients, lambda_out device float n_blocks (may be NULL), obj_out as
 * in csv_decode_gop (may be NULL). */
int csv_recover_blocks(csv_ctx* ctx, const csv_params* p, int32_t n_blocks,
                       const int8_t* codes, const uint8_t* exps, float* s_out,
                       float* lambda_out, double* obj_out, void* stream);

/* ------------------------------------------------------ graph replay */
/* Capture the decode of a fixed batch (same arguments as csv_decode_batch)
 * into a HIP graph: one eager decode first builds every per-stream operator
 * and sizes the context's scratch, then the whole sequence (key frames,
 * dequantisation, lambda, the persistent fused recovery launch with its
 * tile table, synthesis, FP64 check) is stream-captured on `stream`
 * (a non-default stream).  csv_graph_launch replays it over whatever the
 * bound input buffers hold at launch time, writing the bound outputs.  The
 * graph keeps using the context's scratch: replays and other decodes on
 * that context must not overlap on the device.  A later call on the same
 * context that needs a larger scratch buffer than the capture sized moves
 * that buffer; csv_graph_launch then returns CSV_EINVAL without launching
 * anything (recapture after such calls, or give them their own context).
 * Destroy the graph before its context. */
typedef struct csv_graph csv_graph;
int csv_graph_capture(csv_ctx* ctx, int32_t count, const csv_params* params,
                      const csv_gop_stream* in, uint8_t* const* frames_out,
                      float* const* cs_float_out, double* const* obj_out, void* stream,
                      csv_graph** out);
int csv_graph_launch(csv_graph* g, void* stream);
int csv_graph_destroy(csv_graph* g);

/* ------------------------------------------------------- measurement */
/* Event timing of named kernel ranges on the stream they run on ("fista_bf16",
 * "fista_fp32", "tv_fp32", "tv_bf16", "tv_whole", "prepare", "synth",
 * "final64", "key_decode", "measure").  While enabled, every such range
 * records a pair of HIP events.  csv_profile_query waits
 * for the recorded events and returns the summed milliseconds and the number
 * of ranges for `name` since the last reset. */
int csv_profile_enable(csv_ctx* ctx, int on);
int csv_profile_query(csv_ctx* ctx, const char* name, double* total_ms, int64_t* launches);
int csv_profile_reset(csv_ctx* ctx);

/* Achievable ceilings of the context's device, from short microbenchmarks
 * (synchronous, about 50 ms; allocates and frees 1 GiB + 2 MiB inside the
 * context budget, CSV_ENOMEM if it does not fit).  A kernel's roofline
 * fraction is read against these as well as against the datasheet peaks:
 *   mfma_bf16_tflops  dense 32x32x16 BF16 MFMA chains on every CU;
 *   l2_read_tbs       every CU streaming the same 1 MiB buffer, which stays
 *                     resident in each XCD's L2 (L2 -> CU read bandwidth);
 *   hbm_read_tbs      one pass over a 1 GiB buffer (HBM read bandwidth);
 *   lds_read_tbs      16-byte LDS reads on every CU.
 * Bandwidths are in 1e12 bytes/s, totals over the whole device. */
typedef struct {
    double mfma_bf16_tflops, l2_read_tbs, hbm_read_tbs, lds_read_tbs;
    int32_t compute_units;
} csv_ceilings;
int csv_probe_ceilings(csv_ctx* ctx, csv_ceilings* out);

#ifdef __cplusplus
}
#endif
#endif /* CSV_H */
