/*
 * csv_config.h - parameter configurator of the coder (the application-aware
 * configurable mechanism of Sections 2-3: the GOP size and the measurement
 * matrix size are chosen on the encoder side for what the application
 * needs, Fig. 6 and Table I).
 *
 * The paper chooses by tracking success rate; the tracker is not part of this
 * library, so the application's requirement is given as a PSNR floor on the
 * decoded video.  For every candidate (G, M) the configurator runs the coder
 * itself (csv_encode_batch / csv_decode_batch) over a calibration clip and
 * measures the result:
 *   - the clip of F frames is cut into consecutive GOPs of G frames; a final
 *     shorter GOP takes the remaining frames (one frame = key frame only);
 *   - total CR = 8 F H W / (key bits + CS bits), from the coded streams;
 *     key CR and CS CR likewise over the key frames and the CS frames;
 *   - PSNR per decoded frame from the exact integer sum of squared errors,
 *     10 log10(255^2 H W / SSE) (99.99 dB for SSE = 0), averaged over all
 *     frames (the Table I column) and over the CS frames alone;
 *   - the choice is the candidate of largest total CR whose all-frame mean
 *     PSNR is at least the floor (ties: the first in candidate order), or
 *     -1 if none meets it.
 * Candidates are ordered G-major: point i is (gops[i / n_m], ms[i % n_m]).
 */
#ifndef CSV_CONFIG_H
#define CSV_CONFIG_H

#include "csv.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t gop, m;
    uint64_t bits_key, bits_cs;      /* over the whole clip */
    double cr_total, cr_key, cr_cs;
    double psnr_all, psnr_cs;        /* mean dB over all frames / over CS frames */
    int32_t meets_floor;
} csv_config_point;

/* Sweep (G, M) over a calibration clip and choose.
 *   base:    every other parameter (size, block, seed, stream, iterations,
 *            precision, flags); base->gop and base->m are ignored;
 *   clip:    device, n_frames x H x W uint8;
 *   gops:    host, n_g GOP sizes (each >= 1); ms: host, n_m values of M
 *            (each 1..n);
 *   points:  host, n_g * n_m results; *best: the chosen index or -1.
 * Synchronous (returns after the sweep; work runs on `stream`).  Uses the
 * context's scratch for the coded streams and decoded frames of one
 * candidate at a time. */
int csv_configure(csv_ctx* ctx, const csv_params* base, const uint8_t* clip, int32_t n_frames,
                  const int32_t* gops, int32_t n_g, const int32_t* ms, int32_t n_m,
                  double psnr_floor, csv_config_point* points, int32_t* best, void* stream);

/* Per-frame sums of squared differences of two device stacks of n_frames
 * H x W uint8 frames, exact, into device uint64 sse[n_frames].  Async. */
int csv_frame_sse(csv_ctx* ctx, const uint8_t* a, const uint8_t* b, int32_t n_frames,
                  int32_t width, int32_t height, uint64_t* sse, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CSV_CONFIG_H */
