/*
 * sketch_serve.h -- request server for sketches of uneven shapes.
 *
 * A server takes a stream of independent sketch requests
 *
 *     Y_r = A_r * Omega(seed_r)[row0_r : row0_r + n_r, col0_r : col0_r + k_r]
 *
 * (the product of sketch_gen_matmul in sketch.h: the local multiplication of
 * Alg. 1 with GenRandom, Sec. 4 and Sec. 6.3) with different m, n and k.  The
 * paper runs one such product per process; serving many of them on one device
 * is this library's addition.  Requests run with continuous batching:
 *   - Admission.  Requests wait in one FIFO queue.  The head is admitted as soon
 *     as an in-flight slot is free and its device-memory footprint (below) fits
 *     in the server's budget; no request overtakes the head.  A request whose
 *     footprint exceeds the whole budget is refused at submission.
 *   - Batching.  Requests admitted together are grouped by kernel class (the
 *     same tile code: storage type, and the sketch-width class of the streaming
 *     kernel or the N-tile count of the matrix-core kernel), up to max_batch per
 *     group, and each group runs as ONE persistent launch: a fixed grid of
 *     workgroups walks the tiles of all its requests (each XCD a contiguous
 *     range), followed by one launch of the FP64 strip sums of all of them.
 *     While at least two batches are in flight, admission waits until half the
 *     slots are free, so that requests arriving under load share launches; an
 *     idle or nearly idle device admits at once.
 *   - Overlap.  Batches go round-robin to a pool of HIP streams, so requests
 *     admitted while others run share the device with them.
 *   - Device residency.  Seeds, offsets and shapes travel in the launch
 *     arguments; the FP32 strip partials and any staged A live in the server's
 *     device arena; nothing returns to the host but completion.
 * Every request runs exactly the tiles, strip boundaries and FP64 summation
 * order of a sketch_gen_matmul call on the same arguments, so its Y is bitwise
 * the same alone, in any batch, and as a direct call.
 *
 * Footprint of a request (bytes of the arena it holds from admission to
 * completion), each part rounded up to 256 B:
 *   - FP32 strip partials: S * m * k * 4 when S > 1 strips (S from
 *     sketch_strip_width(a_dtype, k)), else 0;
 *   - staged A for SK_SRC_HOST and SK_SRC_SYNTH: m * ld * size(a_dtype), with
 *     ld = n rounded up to 16 bytes.
 *
 * Threads: one worker thread per server launches batches and polls their
 * completion events; every function below may be called from any host thread.
 * The server runs on the device that is current when it is created.
 * Ordering: the server's streams are not ordered after the caller's streams.
 * A request's input must be complete when it is submitted (e.g. the stream
 * that wrote it synchronised), and its Y may be read once the ticket reports
 * SK_REQ_DONE.
 */
#ifndef SKETCH_SERVE_H
#define SKETCH_SERVE_H

#include "sketch.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Where a request's A comes from. */
enum sk_source {
    SK_SRC_DEVICE = 0,   /* A is caller device memory (as in sketch_gen_matmul)          */
    SK_SRC_HOST = 1,     /* A is caller host memory (pinned for overlap), copied into the
                            arena at admission                                           */
    SK_SRC_SYNTH = 2     /* synthetic load: the server fills an arena A (FP32) at
                            admission with A(i, j) ~ N(0,1): Box-Muller (hardware log2,
                            sin, cos, sqrt) on word (j mod 4) of Philox4x32-10 at counter
                            (j div 4, i, 0, 1) under key a_seed; deterministic on a given
                            device, not bit-specified.  A must be NULL                   */
};

enum sk_req_state {
    SK_REQ_QUEUED = 0,
    SK_REQ_RUNNING = 1,   /* admitted: memory held, work enqueued */
    SK_REQ_DONE = 2,      /* Y written                            */
    SK_REQ_FAILED = 3,    /* launch error (status holds it)       */
    SK_REQ_CANCELLED = 4
};

typedef struct sk_request {
    int a_source;            /* sk_source                                             */
    int a_dtype;             /* sk_adtype; SK_A_F32 for SK_SRC_SYNTH                   */
    const void* A;           /* see sk_source; 16-B aligned with lda*size % 16 == 0
                                for SK_SRC_DEVICE                                      */
    int64_t m, n, lda;       /* m, n >= 1; lda >= n (ignored for SK_SRC_SYNTH)         */
    const float* a_scales;   /* device, ceil(m/128) scales for SK_A_FP8_E4M3, else NULL */
    uint64_t a_seed;         /* SK_SRC_SYNTH only                                      */
    uint64_t seed;           /* Omega's seed                                           */
    int64_t omega_row0, omega_col0;
    int64_t k;               /* 1 <= k <= 1024                                         */
    void* Y;                 /* device, m x k, leading dim ldy >= k                    */
    int y_dtype;             /* sk_ydtype                                              */
    int64_t ldy;
    int beta;                /* 0: Y = A*Omega; 1: Y += A*Omega                        */
    int omega_dist;          /* sk_dist of Omega (0 = normal)                          */
} sk_request;

/* Times are microseconds on the server's host clock (0 = its creation). */
typedef struct sk_ticket_info {
    int state;               /* sk_req_state                                          */
    int status;              /* SK_OK, or the error of a failed request               */
    int64_t batch;           /* id of the batch that ran it (0 before admission)      */
    int batch_size;          /* requests in that batch                                */
    size_t footprint;        /* arena bytes held while admitted                       */
    double t_submit_us;      /* submission                                            */
    double t_admit_us;       /* admission (memory and slot granted, work enqueued)    */
    double t_done_us;        /* completion seen by the worker                         */
    double stage_us;         /* device time of the batch's A staging (copy / fill)    */
    double sketch_us;        /* device time of the batch's sketch and strip sums      */
} sk_ticket_info;

typedef struct sk_serve_stats {
    int64_t submitted, admitted, completed, failed, cancelled, rejected;
    int64_t batches, queued, running, max_running;
    size_t budget_bytes, bytes_in_use, peak_bytes_in_use;
} sk_serve_stats;

typedef struct sk_server sk_server;

/* Footprint of a request under the rule above; 0 for an invalid request. */
size_t sk_request_footprint(const sk_request* r);

/*
 * Create a server on the current device: allocates the arena (budget_bytes,
 * may be 0) once, n_streams HIP streams (default priority) and the worker.
 *   max_slots  requests in flight at once (>= 1);
 *   max_batch  requests per launch, 1 .. 16;
 *   n_streams  1 .. 8.
 * SK_ENOMEM if the arena cannot be allocated, SK_EHIP for other runtime errors.
 */
int sk_server_create(size_t budget_bytes, int max_slots, int max_batch, int n_streams,
                     sk_server** out);

/*
 * Queue a request (copied; the buffers it points to must stay valid, and Y
 * untouched, until the request is done, failed or cancelled).  On success
 * *ticket > 0.  Argument errors as for sketch_gen_matmul (plus SK_EINVAL for
 * m, n or k == 0, or a bad source), SK_EBUDGET if the footprint exceeds the
 * budget, SK_EQUEUE if the queue (4096 requests) is full.
 */
int sk_server_submit(sk_server* s, const sk_request* r, int64_t* ticket);

/* State and timings of a ticket; SK_EQUEUE for an unknown (or forgotten)
 * ticket.  The server keeps the records of its 65536 most recent finished
 * requests. */
int sk_server_poll(sk_server* s, int64_t ticket, sk_ticket_info* info);

/* Block until the ticket is done, failed or cancelled (SK_OK, info filled) or
 * timeout_s seconds have passed (SK_ETIMEOUT; timeout_s < 0 waits forever). */
int sk_server_wait(sk_server* s, int64_t ticket, double timeout_s, sk_ticket_info* info);

/* Cancel a request that is still queued (SK_OK); SK_EQUEUE otherwise. */
int sk_server_cancel(sk_server* s, int64_t ticket);

/* Counters since creation, and the arena bytes in use now and at peak. */
int sk_server_stats(sk_server* s, sk_serve_stats* out);

/* Current time on the server's clock, microseconds. */
double sk_server_now_us(sk_server* s);

/* Cancel what is queued, wait for what runs, free the arena, streams and
 * worker.  The handle is invalid afterwards. */
int sk_server_destroy(sk_server* s);

#ifdef __cplusplus
}
#endif
#endif /* SKETCH_SERVE_H */
