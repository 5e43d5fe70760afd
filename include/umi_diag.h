/*
 * umi_diag.h -- measurement aids of the MI355X UMI library (libumi_diag.so).
 * Nothing here is part of the method; benchmarks use it to report the
 * device's sustained FP32 rate beside the published peak.
 */
#ifndef UMI_DIAG_H
#define UMI_DIAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * umi_diag_fma_peak -- launch `grid` workgroups of 256 threads, each thread
 * running `iters` rounds of 16 independent scalar FP32 fused multiply-adds
 * (no packed forms), on `stream` (a hipStream_t).  out: device float32
 * [grid * 256], written once per thread (keeps the work live).  *flop (host,
 * may be NULL) receives the FLOPs the launch performs (2 per FMA).  Returns 0,
 * 1 for a bad argument (nothing launched), 3 for a launch error.  Time it
 * with events on the same stream.
 */
int32_t umi_diag_fma_peak(int64_t iters, int32_t grid, float* out, void* stream,
                          double* flop);

#ifdef __cplusplus
}
#endif

#endif /* UMI_DIAG_H */
