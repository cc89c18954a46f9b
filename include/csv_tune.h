/*
 * csv_tune.h - tile-shape autotuner of the fused recovery kernel.
 *
 * The fused BF16 recovery kernel (csv.h, precision CSV_BF16) is compiled in
 * a few variants per (n = block^2, M rounded up to 32) class: column tiles
 * of 32 blocks per workgroup, operator prefetch ring depths and the number
 * of iterate tiles kept in LDS.  The tuner times each variant on a fixed
 * synthetic operator and synthetic codes and makes the fastest the class's
 * choice for every later decode in this process.
 */
#ifndef CSV_TUNE_H
#define CSV_TUNE_H

#include "csv.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Time every variant of the class of (block, m) on n_blocks synthetic
 * blocks with `iters` FISTA iterations: after about 150 ms of launches of
 * the current choice (so that no variant is timed on idle clocks), every
 * variant is timed in two interleaved rounds, each the median of 3
 * launches, and keeps its faster round.
 * ms_out (may be NULL) receives one time per variant (at most 8 entries);
 * *count the number of variants, *best the chosen index.  If json_path is
 * non-empty the choices of all classes are written there as JSON.
 * Synchronous. */
int csv_autotune(csv_ctx* ctx, int32_t block, int32_t m, int32_t iters, int32_t n_blocks,
                 const char* json_path, double* ms_out, int32_t* count, int32_t* best);

/* Apply the choices recorded in a file written by csv_autotune
 * (CSV_ENOTFOUND if unreadable, CSV_EINVAL if it names no known variant). */
int csv_autotune_load(const char* json_path);

/* Report the current choice of the class of (block, m). */
int csv_autotune_choice(int32_t block, int32_t m, char* name, size_t name_len, int32_t* index,
                        int32_t* count);

/* Make variant `index` the choice of the class of (block, m). */
int csv_autotune_set(int32_t block, int32_t m, int32_t index);

#ifdef __cplusplus
}
#endif
#endif /* CSV_TUNE_H */
