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

#ifdef __cplusplus
}
#endif

#endif /* UMI_SERVE_H */
