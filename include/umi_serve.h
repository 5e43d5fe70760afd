/*
 * umi_serve.h -- host-side helper of the UMI serving loop (libumi.so).
 *
 * Not a step of the method (arXiv 2604.06602, Section 2): the serving loop
 * batches many curves per device step, and each step stages every curve's
 * flux and time into pinned host memory before one host-to-device copy, and
 * copies each result back out of pinned memory afterwards.  Done curve by
 * curve from an interpreter, those copies cost more in per-call overhead and
 * lock hand-offs than in bytes moved; these entry points do a whole list of
 * them in one call: host-to-host copies split over a small pool of native
 * threads, and host/device copies enqueued on a stream.
 */
#ifndef UMI_SERVE_H
#define UMI_SERVE_H

#include <stdint.h>

#include "umi.h"

#ifdef __cplusplus
extern "C" {
#endif

#define UMI_HOST_COPY_MAX_THREADS 64

/* Host-to-host copies: for i in [0, n), bytes[i] bytes from src[i] to dst[i].
 * All pointers, including the three arrays themselves, are [host] memory
 * (pageable or pinned) owned by the caller; no device memory and no stream are
 * involved, and the call returns when every copy is complete.  The copies are
 * cut into pieces of at most 1 MiB, which up to `threads` threads (the calling
 * thread and threads - 1 pool threads, started on first use and kept for the
 * life of the process) take in turn.  The regions of different copies must not
 * overlap (the result is then undefined, as for memcpy).  Calls from several
 * threads are safe: those that use the pool take it one after another, and a
 * call with one piece, or with threads = 1, copies on the calling thread.
 * Errors: n < 0, threads < 1 or > UMI_HOST_COPY_MAX_THREADS, a NULL array with
 * n > 0, a negative size, or a NULL pointer with a positive size give
 * UMI_ERR_INVALID_ARG before anything is copied.  n = 0 is a no-op. */
umi_status umi_host_copy_many(void* const* dst, const void* const* src, const int64_t* bytes,
                              int64_t n, int32_t threads);

#define UMI_COPY_H2D 1
#define UMI_COPY_D2H 2
#define UMI_COPY_KERNEL 4 /* or-ed into kind: see umi_copy_async */

/* Asynchronous host/device copies on `stream` (a hipStream_t, NULL = the
 * legacy default stream): for i in [0, n), bytes[i] bytes from src[i] to
 * dst[i], host to device when kind is UMI_COPY_H2D and device to host when it
 * is UMI_COPY_D2H, enqueued in order.  The three arrays are [host] and read
 * before the call returns; the host side of each copy should be pinned memory
 * (hipHostMalloc), or the runtime may complete the copy before returning.  The
 * caller keeps every buffer alive, and the host buffers untouched, until the
 * stream work completes.  For the serving loop: the copies of a whole step in
 * one call.
 * With UMI_COPY_KERNEL or-ed into kind, the copies run as a kernel on
 * `stream` (one launch per 64 copies, one workgroup per 32 KiB piece) that
 * reads and writes the host buffers directly over the bus, instead of being
 * handed to the runtime's copy engines, whose enqueue has been seen to block
 * the calling thread for several milliseconds now and then.  The host side
 * of every copy must then be pinned memory from hipHostMalloc (as torch's
 * pinned tensors are), which the device reaches at its host address;
 * pageable memory is not allowed on this path.  Copies of one call must not
 * overlap.
 * Errors: n < 0, an unknown kind, a NULL array with n > 0, a negative size or
 * a NULL pointer with a positive size give UMI_ERR_INVALID_ARG before anything
 * is enqueued; a failing enqueue gives UMI_ERR_DEVICE (copies before it stay
 * enqueued).  n = 0 is a no-op. */
umi_status umi_copy_async(void* const* dst, const void* const* src, const int64_t* bytes,
                          int64_t n, int32_t kind, void* stream);

/*
 * Native serving loop.  A server owns one device's resident arena (flux f32,
 * time f64 and trend f32 arrays of `capacity` samples), a replayable plan over
 * it, pinned staging rings, three streams (uploads, steps, downloads), a
 * scheduler thread and a waiter thread.  Requests -- one light curve each,
 * with its own W, alpha and c (Section 2; the Table 4 settings mix freely in
 * one step) -- are admitted first-in first-out while their samples fit the
 * arena (each admission group gets one contiguous range), staged into pinned
 * memory and uploaded by the copy kernel, and run as continuous-batching
 * steps: every uploaded group with the same iteration count joins the next
 * step, up to max_curves curves and max_step_samples samples, with up to
 * max_inflight steps on the device at once.  When a step's device work is
 * done the waiter thread copies its trends straight into each request's
 * `out` buffer and reports the requests complete.
 *
 * umi_server_submit queues a request and returns at once.  flux [n] float32,
 * time [n] float64 (or NULL: no gap breaks) and out [n] float32 are [host]
 * memory the caller owns and keeps alive, unchanged (flux, time) and
 * untouched (out), until the request is reported complete; `tag` is the
 * caller's identifier, returned with the completion.  `arrival` is the
 * request's arrival time in seconds of CLOCK_MONOTONIC (Python's
 * time.perf_counter on Linux), or a negative value for "now"; latency
 * figures run from it.  n = 0 completes at once.  Errors (nothing queued, no
 * completion reported): W even, < 1 or > max_W, alpha or c not finite and
 * > 0, iters < 0, n < 0 or n > capacity, a NULL flux or out with n > 0, or a
 * server that is shutting down give UMI_ERR_INVALID_ARG.  Safe from any
 * number of threads.
 *
 * umi_server_poll waits up to timeout_s seconds (0: no wait) for completions
 * and moves at most `max` of them, oldest first, into out[], setting *n_out.
 * A completion's status is UMI_OK when `out` holds the trend, else the error
 * of the step the request ran in (its `out` is then unspecified).
 *
 * umi_server_shutdown finishes every queued request, stops the scheduler and
 * frees the device and pinned memory; completions stay available to
 * umi_server_poll.  umi_server_destroy shuts down (if not done yet) and frees
 * the server.  umi_server_stats_get fills *out with counters since creation or
 * the last umi_server_reset_stats.
 *
 * Errors of umi_server_create: a config field out of range gives
 * UMI_ERR_INVALID_ARG; device or pinned memory that cannot be allocated gives
 * UMI_ERR_NO_MEMORY; a runtime error UMI_ERR_DEVICE.  A failure inside the
 * scheduler thread fails every request not yet launched with UMI_ERR_DEVICE
 * (launched steps still complete) and stops it; later submits give
 * UMI_ERR_INVALID_ARG.
 */
typedef struct umi_server umi_server;

typedef struct {
    int64_t capacity;         /* arena samples (> 0) */
    int64_t max_step_samples; /* samples per step and admission group (0: 2^22); a
                                 lone larger request runs as a step of its own;
                                 it bounds how long a step's result copies take
                                 when a backlog has built up */
    int64_t staging_bytes;    /* pinned upload ring (0: 4 GiB); the download ring
                                 is a third of it */
    int32_t max_curves;       /* curves per step (0: 4096) */
    int32_t max_W;            /* largest W of any request (0: 721) */
    int32_t max_inflight;     /* steps on the device at once (0: 2) */
    int32_t copy_threads;     /* threads of the staging copies (0: 4) */
    int32_t device;           /* HIP device */
    int32_t reserved;         /* must be 0 */
} umi_server_config;

typedef struct {
    uint64_t tag;
    int32_t status;           /* umi_status */
    int32_t reserved;
    double admitted;          /* CLOCK_MONOTONIC seconds: range allocated */
    double launched;          /* its step enqueued */
    double done;              /* result in `out` */
} umi_server_completion;

typedef struct {
    int64_t submitted, completed, failed, rejected;
    int64_t steps, step_curves, samples, largest_step_samples;
    int64_t arena_capacity, arena_used, arena_high_water;
    int64_t staging_fallbacks;  /* one-off pinned blocks for oversize groups */
    double loop_s[4];           /* seconds finishing steps (waiter thread), then
                                   admitting, uploading, launching (scheduler) */
    double longest_iteration_s; /* longest scheduler iteration */
    double longest_iteration_loop_s[4];  /* its split as loop_s ([0] is 0) */
    double exec_s[4];           /* staging copy, upload enqueue, plan run, result copy */
} umi_server_stats;

umi_status umi_server_create(const umi_server_config* config, umi_server** out);
umi_status umi_server_submit(umi_server* server, const float* flux, const double* time,
                             int64_t n, int32_t W, float alpha, float c, int32_t iters,
                             double arrival, float* out, uint64_t tag);
umi_status umi_server_poll(umi_server* server, umi_server_completion* out, int32_t max,
                           double timeout_s, int32_t* n_out);
umi_status umi_server_stats_get(umi_server* server, umi_server_stats* out);
umi_status umi_server_reset_stats(umi_server* server);
umi_status umi_server_shutdown(umi_server* server);
umi_status umi_server_destroy(umi_server* server);

#ifdef __cplusplus
}
#endif

#endif /* UMI_SERVE_H */
