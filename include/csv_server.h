/*
 * csv_server.h - continuous-batching decode server over the csv.h coder.
 *
 * Streams (cameras) are registered once: their measurement operator,
 * step constant and fragment layouts become resident in device memory
 * (Section 3.1: one random matrix per stream; Section 2: the GOP size and
 * matrix size are per-stream configuration).  GOP decode requests
 * (Section 3.2) are then submitted as they arrive.  A worker thread admits
 * requests while the device-memory budget allows, groups the admitted ones
 * into batches, and launches each batch (key frames, dequantisation,
 * lambda, one fused recovery launch over all their blocks, synthesis) on one
 * of several HIP streams, so that a batch formed while another runs
 * overlaps with it on the device.  Latency is completion time minus the
 * caller's arrival time, on the csv_clock() clock.
 *
 * Ownership: the GOP stream buffers passed to csv_submit are caller-owned
 * device memory whose contents must be complete when csv_submit is called
 * and must stay valid until the request completes (or is cancelled).
 * Decoded frames live in server memory until csv_poll copies them out.
 * Thread safety: every entry point may be called from any host thread.
 */
#ifndef CSV_SERVER_H
#define CSV_SERVER_H

#include "csv.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct csv_server csv_server;

enum {
    CSV_SERVER_FAKE_EXECUTOR = 1   /* test hook: host-only executor, no device work */
};

typedef struct {
    size_t mem_budget;          /* device bytes charged to requests (0: 4 GiB): an admitted or
                                   running request holds its decoded frames plus the recovery
                                   working set of its path (coefficients, y^, lambda and its
                                   adjoint; the FP32 iterates and TV state where used); a
                                   finished one holds only its frames, until csv_poll or
                                   csv_cancel releases them.  Admission control only: resident
                                   operators and the batch slots' grow-only scratch are not
                                   charged (csv_stats.device_bytes reports them) */
    int32_t max_queue;          /* waiting requests beyond which csv_submit returns CSV_EAGAIN (0: 4096) */
    int32_t max_batch_blocks;   /* recovery blocks per batch (0: 262144) */
    int32_t precision;          /* CSV_BF16 or CSV_FP32 for every request */
    int32_t hip_streams;        /* streams used by consecutive batches, 1..4 (0: 2) */
    int32_t flags;              /* CSV_SERVER_* */
    double fake_us_per_block;   /* fake executor: service time per recovery block */
    double fake_fail_every;     /* fake executor: fail every k-th batch (0: never) */
} csv_server_opts;

/* Statistics since server creation or the last csv_server_reset_stats.
 * Completion counts, pixels and latencies cover only requests submitted
 * since then (a request submitted earlier that completes later is left out
 * of them, e.g. warm-up requests). */
typedef struct {
    uint64_t submitted, admitted, completed, rejected, cancelled, failed;
    uint64_t recovered_pixels;  /* CS pixels of completed requests */
    double p50_ms, p99_ms, mean_ms, max_ms;   /* completed requests */
    double mpix_per_s;          /* recovered pixels / (last completion - first arrival) */
    size_t bytes_in_flight, peak_bytes;   /* charged against mem_budget */
    int32_t queue_depth;        /* waiting, not yet admitted */
    int32_t batches;            /* batches launched */
    int32_t max_concurrent;     /* most batches in flight at once */
    double first_arrival_s;     /* csv_clock() of the first counted arrival (-1: none) */
    double last_done_s;         /* csv_clock() of the last counted completion */
    size_t device_bytes;        /* device memory the server holds, as of the latest batch
                                   launch: resident operators, the batch slots' grow-only
                                   scratch and the output pool; unlike bytes_in_flight this
                                   is not bounded by mem_budget */
} csv_stats;

/* Monotonic clock in seconds (the server's latency clock). */
double csv_clock(void);

int csv_server_create(int device, const csv_server_opts* opts, csv_server** out);
/* Waits for in-flight batches, frees everything. */
int csv_server_destroy(csv_server* srv);

/* Register a stream: validates p (precision is taken from the server),
 * builds its operator (measurement matrix, A, step constant) synchronously
 * and returns its id.  CSV_EUNSUPPORTED when the server's precision has no
 * recovery for the stream: a BF16 server needs a fused kernel for its block
 * size and M (for CSV_FLAG_TV: 16 x 16 blocks, M up to 128); whole-frame
 * streams (CSV_FLAG_WHOLE_FRAME) need an FP32 server and CSV_FLAG_TV. */
int csv_server_register_stream(csv_server* srv, const csv_params* p, uint32_t* sid);
/* Register `count` streams at once (params and sids: host arrays of count
 * entries): the same validation and ids as count single registrations (in
 * order; none is registered if any is refused), with the new operators'
 * FP64 power iterations for M <= 320 run side by side, one workgroup per
 * stream and one launch per size class (M up to 32, 64, 128, 256, 320), so
 * that the setup of many cameras costs about as much as the slowest of
 * them; operators with larger M run their many-workgroup power iterations
 * one after another. */
int csv_server_register_streams(csv_server* srv, int32_t count, const csv_params* params,
                                uint32_t* sids);

/* Submit one GOP of stream sid.  t_arrival: csv_clock() seconds (<= 0:
 * now).  Returns CSV_EAGAIN if the waiting queue is full, CSV_ENOMEM if the
 * request alone exceeds the budget, CSV_ENOTFOUND for an unknown sid. */
int csv_submit(csv_server* srv, uint32_t sid, const csv_gop_stream* in, double t_arrival,
               uint64_t* ticket);

/* Poll a ticket.  *done = 1: the decoded G x H x W frames were copied to
 * frames_out (device memory, may be NULL to discard) and the ticket is
 * released; *done = 0: still pending.  Returns CSV_ECANCELED, CSV_ENOTFOUND,
 * or the request's failure code (the ticket is released then too). */
int csv_poll(csv_server* srv, uint64_t ticket, uint8_t* frames_out, int32_t* done);

/* Cancel a ticket: a waiting request is dropped at once; one already on
 * the device is discarded when its batch ends. */
int csv_cancel(csv_server* srv, uint64_t ticket);

/* Block until nothing waits or runs.  Returns CSV_EAGAIN when timeout_s
 * elapses, and at once when the queue can make no progress: nothing runs and
 * the next waiting request does not fit the budget left by finished requests
 * that were not polled (poll or cancel them, then drain again). */
int csv_server_drain(csv_server* srv, double timeout_s);

int csv_server_stats(csv_server* srv, csv_stats* out);
/* Start a new statistics window: counters, latencies and rates restart
 * from zero; requests already submitted are not counted when they finish. */
int csv_server_reset_stats(csv_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* CSV_SERVER_H */
