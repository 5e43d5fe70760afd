/*
 * umi.h -- C ABI of the MI355X (gfx950) UMI detrending library.
 *
 * UMI (arXiv 2604.06602, Section 2) computes, at every sample of a light
 * curve, a robust location estimate over a window of W samples centred on it:
 *   Phase 1 (Section 2.1)        the exact window median;
 *   Phase 2 (Section 2.2, Eq. 1) the upper-RMS scale s = 0.6745 * sigma_upper
 *                                from the points strictly above the median;
 *   Phase 3 (Section 2.3, Eqs. 2-4) `iters` asymmetric Tukey-bisquare
 *                                re-weightings with residuals below the
 *                                location scaled by alpha, u = (x - mu)/(c s).
 * The estimate is the "trend"; Section 2 also fixes W = round(0.5/dt) | 1.
 *
 * Conventions fixed by this library (where the paper is silent):
 *   - the window is the sample-index window [i-h, i+h], h = (W-1)/2, cut at the
 *     ends of the sample's segment; invalid samples inside it are skipped;
 *   - a sample is valid when its flux is finite and, if a time array is given,
 *     its time is finite;
 *   - a new segment starts where consecutive valid times differ by more than
 *     UMI_GAP_DAYS (strictly); with no time array there are no breaks;
 *   - a segment with fewer than max(1, floor(W/3)) valid samples (the minimum
 *     segment length scaled to W/3, Section 4.4) gives NaN;
 *   - the median is the lower median (0-based rank floor((n-1)/2)) in IEEE-754
 *     totalOrder of the float32 bits, returned bit-exact;
 *   - if no point lies strictly above the median the scale is 0 and the trend
 *     is the median; iters = 0 returns the median.
 * Arithmetic is float32 on the GPU.
 *
 * Memory and streams.  Every array argument is a DEVICE pointer owned by the
 * caller unless marked [host].  Calls are asynchronous on `stream` (a
 * hipStream_t, NULL = the legacy default stream): they validate on the host,
 * enqueue work and return without synchronising.  The caller keeps every
 * buffer alive until that stream work completes.  The library keeps a
 * workspace per (device, stream), grown on demand and freed by umi_release();
 * it retains no caller pointer after a call returns.
 *
 * Packed ragged batches.  Curve b occupies samples [off_b, off_b + lengths[b])
 * of every per-sample array, where off is the exclusive prefix sum of lengths.
 *
 * Errors.  Functions return a umi_status and never throw.  Arguments are
 * checked before anything is enqueued; on UMI_ERR_INVALID_ARG and
 * UMI_ERR_UNSUPPORTED nothing is written.  umi_last_error() returns a
 * thread-local message for the last failing call on the calling thread.
 * NaN outputs at invalid samples or dead segments are data, not errors.
 */
#ifndef UMI_H
#define UMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UMI_GAP_DAYS 0.5     /* segment break threshold in days */
#define UMI_MAX_WINDOW 2047  /* largest supported W */

typedef enum {
    UMI_OK = 0,
    UMI_ERR_INVALID_ARG = 1, /* bad argument; nothing enqueued */
    UMI_ERR_NO_MEMORY = 2,   /* workspace could not be allocated */
    UMI_ERR_DEVICE = 3,      /* a HIP runtime or launch error */
    UMI_ERR_UNSUPPORTED = 4  /* valid but outside the library's limits (W) */
} umi_status;

/* Launch modes of the batch call. */
typedef enum {
    UMI_MODE_PERSISTENT = 0, /* one launch for the whole batch: a grid of
                                long-lived workgroups pops cost-sorted tiles
                                from a device work queue (default) */
    UMI_MODE_PER_CURVE = 1   /* one launch per curve (comparison mode) */
} umi_mode;

/* Tuning knobs; zero in a field means "use the library's choice" (its
 * built-in defaults, or the tuning table loaded with umi_set_tuning).  With
 * tile = 0, a batch that the chosen tiles would cut into fewer tiles than the
 * device has compute units runs with tiles of at most 1024, 512, 256, 128,
 * then 64 output positions, so that more of the chip shares it.  Tiles of
 * more than 256 positions give each window one lane and results that do not
 * depend on the tile size; tiles of at most 256 split every window over 2,
 * 4 or 8 lanes (kept in step by cross-lane sums), which orders the sums
 * differently: such results agree with the others to float32 rounding and
 * are themselves deterministic. */
typedef struct {
    int32_t mode;          /* umi_mode */
    int32_t tile;          /* output positions per tile (0 = auto) */
    int32_t groups_per_cu; /* persistent workgroups per compute unit (0 = auto) */
    int32_t reserved;      /* must be 0 */
    void* main_start;      /* optional hipEvent_t recorded on the stream just
                              before the main (estimate) kernel(s) */
    void* main_stop;       /* optional hipEvent_t recorded just after them */
} umi_launch;

/* Phase 2 scale estimators. */
typedef enum {
    UMI_SCALE_UPPER_RMS = 0, /* the method: s = 0.6745 * sigma_upper from the
                                points strictly above the median (Section 2.2,
                                Eq. 1) */
    UMI_SCALE_MAD = 1        /* ablation: s = the standard MAD, the lower
                                median (rank floor((n-1)/2)) of |x - m| over
                                the window, unscaled (it equals 0.6745 sigma
                                at the Gaussian model); the scale Sections 1
                                and 2.2 contrast with the upper-RMS one and
                                Section 3.1 compares against it */
} umi_scale;

/* Extra options of the _ex calls.  NULL (or all fields zero) is the method
 * as published with the call's alpha and c for every curve. */
typedef struct {
    const float* alpha;  /* [host] n_curves per-curve asymmetry factors, or
                            NULL for the call's alpha.  The use-case settings
                            of Table 4 (planet search 2/5, high-precision
                            3/5, variable stars 1/5, maximum shallow
                            sensitivity 10/2.5) can be mixed in one batch. */
    const float* c;      /* [host] n_curves per-curve c, or NULL */
    int32_t scale;       /* umi_scale */
    int32_t reserved;    /* must be 0 */
    float* detrended;    /* device out, or NULL: flux / trend at every sample
                            of every curve (the normalisation stage Table 3
                            lists), laid out like trend; NaN where the trend
                            is NaN.  float32 division, correctly rounded. */
    const double* window_days; /* [host] n_curves per-curve window lengths in
                            days, or NULL.  A value > 0 makes that curve's
                            windows time windows (the window_length of
                            Section 4.2, for irregular cadence): sample i's
                            window keeps the valid samples j of its W-sample
                            index window with |t_j - t_i| <= window_days / 2
                            (float64), so W must be at least the largest
                            number of samples such a window can hold.  Needs
                            `time`, non-decreasing over each curve's valid
                            samples (otherwise results are unspecified).  0 =
                            the index window; negative or non-finite values
                            give UMI_ERR_INVALID_ARG. */
} umi_options;

/*
 * umi_detrend -- one curve (Section 2; gap handling per Section 4.4).
 *   flux   [n] float32 fluxes.
 *   time   [n] float64 times in days, or NULL for no gap breaks.
 *   n      number of samples (>= 0; 0 is a no-op).
 *   W      window in samples: odd, 1 <= W <= UMI_MAX_WINDOW.
 *   alpha  asymmetry factor for residuals below the location (> 0, finite);
 *          2 is the paper's default, 1 the symmetric biweight.
 *   c      bisquare tuning constant (> 0, finite); the paper uses 5.
 *   iters  number of re-weighting iterations (>= 0); the paper uses 5.
 *   trend  [n] float32 out: the location estimate, NaN at invalid samples and
 *          in dead segments.
 *   median [n] float32 out (may be NULL): the window median, bit-exact.
 *   stream hipStream_t to enqueue on.
 * Same as umi_detrend_batch with one curve.
 */
umi_status umi_detrend(const float* flux, const double* time, int64_t n,
                       int32_t W, float alpha, float c, int32_t iters,
                       float* trend, float* median, void* stream);

/*
 * umi_detrend_batch -- a packed ragged batch of curves in one call.
 *   flux, time, trend, median  as for umi_detrend, over sum(lengths) samples.
 *   lengths  [host] n_curves sample counts (>= 0).
 *   n_curves number of curves (>= 0; 0 is a no-op).
 *   W        [host] n_curves odd window sizes, one per curve.
 *   alpha, c, iters  as for umi_detrend, shared by all curves.
 *   launch   [host] launch options, or NULL for the defaults.
 * The call copies the tile list it builds to the device from a pinned
 * staging buffer; `lengths` and `W` may be reused as soon as it returns.
 */
umi_status umi_detrend_batch(const float* flux, const double* time,
                             const int64_t* lengths, int64_t n_curves,
                             const int32_t* W, float alpha, float c,
                             int32_t iters, float* trend, float* median,
                             const umi_launch* launch, void* stream);

/*
 * umi_detrend_gather -- like umi_detrend_batch, but curve b sits at samples
 * [offsets[b], offsets[b] + lengths[b]) of every per-sample array instead of
 * back-to-back, so curves resident anywhere in a device arena are batched
 * without copies.
 *   offsets  [host] n_curves sample offsets (>= 0); the ranges must not
 *            overlap (UMI_ERR_INVALID_ARG otherwise).
 * Samples outside every range are neither read nor written.
 */
umi_status umi_detrend_gather(const float* flux, const double* time,
                              const int64_t* offsets, const int64_t* lengths,
                              int64_t n_curves, const int32_t* W, float alpha,
                              float c, int32_t iters, float* trend,
                              float* median, const umi_launch* launch,
                              void* stream);

/*
 * umi_detrend_gather_ex -- umi_detrend_gather with umi_options (per-curve
 * alpha and c, the scale estimator, a detrended-flux output).  `offsets` may
 * be NULL: the curves are then packed back to back as for umi_detrend_batch.
 * Per-curve alpha and c must be finite and > 0 (UMI_ERR_INVALID_ARG
 * otherwise); `alpha` and `c` arguments of the call are still checked and
 * used for any field of `options` that is NULL.
 */
umi_status umi_detrend_gather_ex(const float* flux, const double* time,
                                 const int64_t* offsets, const int64_t* lengths,
                                 int64_t n_curves, const int32_t* W,
                                 float alpha, float c, int32_t iters,
                                 float* trend, float* median,
                                 const umi_options* options,
                                 const umi_launch* launch, void* stream);

/*
 * Plans: a replayable launch over fixed device arrays, for serving loops.
 * umi_plan_create binds the arrays (each `capacity` samples; time and median
 * may be NULL) and a non-default stream, allocates the plan's workspace once
 * and captures its hipGraphs: per staging slot one for batches of at most 256
 * pre-pass chunks (512k samples) and one for any batch, each a copy of the
 * staged tile table, the segmentation pre-pass and the persistent estimate
 * kernel.  umi_plan_run stages one batch -- curves at explicit offsets inside
 * the arrays, as for umi_detrend_gather, at most `max_curves` curves with
 * W <= max_W -- into one of two pinned staging slots and replays that slot's
 * graph for the batch's size on the plan's stream.
 * It allocates no device or pinned memory and returns without synchronising,
 * except that it waits for the replay that used the same slot two calls earlier.  Results
 * of a run are in `trend` / `median` once the stream reaches that point.
 * Calls on one plan are serialised; a plan is used from one device.
 * umi_plan_destroy waits for the stream and frees everything.
 * The same errors as umi_detrend_gather apply; a batch that exceeds the plan
 * (curves, capacity, max_W, tiles) gives UMI_ERR_INVALID_ARG or
 * UMI_ERR_UNSUPPORTED and launches nothing.
 */
typedef struct umi_plan umi_plan;

umi_status umi_plan_create(umi_plan** out, int64_t capacity,
                           int64_t max_curves, int32_t max_W,
                           const float* flux, const double* time,
                           float* trend, float* median, void* stream);
umi_status umi_plan_run(umi_plan* plan, const int64_t* offsets,
                        const int64_t* lengths, const int32_t* W,
                        int64_t n_curves, float alpha, float c, int32_t iters);
/* umi_plan_run with umi_options: the per-curve parameters, scale estimator
 * and detrended output travel with the staged batch, so one captured graph
 * serves them all.  A detrended array must hold the plan's capacity. */
umi_status umi_plan_run_ex(umi_plan* plan, const int64_t* offsets,
                           const int64_t* lengths, const int32_t* W,
                           int64_t n_curves, float alpha, float c,
                           int32_t iters, const umi_options* options);
umi_status umi_plan_destroy(umi_plan* plan);

/*
 * umi_detrend_batch_noalloc -- umi_detrend_batch for callers that cannot
 * allocate memory during the call: code under hipGraph stream capture, tight
 * serving loops, and harnesses that forbid hipMalloc.  Same arguments, layout,
 * results (bit for bit, given the same launch options) and errors as
 * umi_detrend_batch; only the workspace differs.
 *
 * The workspace -- the staged header and curve table, the queue and pre-pass
 * counters, the pre-pass chunk records, the tile list and one segment word
 * per sample -- lives in a static device array
 * of UMI_NOALLOC_SCRATCH_BYTES (about 74 MiB) that each GPU the library runs
 * on holds from the first call on that GPU until the process ends.  A call
 * allocates no device, pinned or host memory on its way to the launches (the
 * curve table is packed into static host arrays and copied with
 * hipMemcpyAsync from pageable memory; only an error message is built on the
 * heap); it looks up the array's device address once per GPU, on that GPU's
 * first call.
 *
 * Limits (larger batches give UMI_ERR_UNSUPPORTED and enqueue nothing):
 *   sum(lengths) <= UMI_NOALLOC_MAX_SAMPLES, n_curves <= UMI_NOALLOC_MAX_CURVES,
 *   and the batch's tiles <= UMI_NOALLOC_MAX_TILES (only windows close to
 *   UMI_MAX_WINDOW, whose tiles are a few positions wide, reach this).
 *
 * Every call on a GPU uses that GPU's one array, whatever the stream, and
 * leaves the last batch's contents there (the kernels overwrite every part
 * they read before reading it; the pre-pass's ticket counters return to zero
 * at the end of each call, and its chunk records carry a launch count that
 * tells them from an earlier call's).  Calls on one stream
 * are ordered by the stream; calls on one GPU whose stream work can overlap
 * (different streams, or several threads) race on the array and give
 * undefined results.  Host-side, concurrent calls are serialised by a lock.
 */
#define UMI_NOALLOC_MAX_SAMPLES 16777216 /* 2^24 samples per call */
#define UMI_NOALLOC_MAX_CURVES 8192
#define UMI_NOALLOC_MAX_TILES 1048576    /* 2^20 tiles per call */
#define UMI_NOALLOC_SCRATCH_BYTES 78250496
umi_status umi_detrend_batch_noalloc(const float* flux, const double* time,
                                     const int64_t* lengths, int64_t n_curves,
                                     const int32_t* W, float alpha, float c,
                                     int32_t iters, float* trend, float* median,
                                     const umi_launch* launch, void* stream);

/* Window-size rule of Section 2: round(window_days / cadence_days) | 1.
 * Returns -1 when either argument is not positive and finite. */
int32_t umi_window_from_cadence(double cadence_days, double window_days);

/* Tuning table: text lines "W_max tile groups_per_cu [samples_max]".  A
 * curve of a batch uses the first line with W <= W_max and, if samples_max
 * is given and > 0, a batch of at most samples_max samples in total; lines
 * are sorted by W_max, then by samples_max, with the lines for any batch
 * size (no or 0 samples_max) last for their W_max.  A batch-size line fixes
 * the tile (tiles of at most 256 positions split each window over 2, 4 or 8
 * lanes); otherwise the small-batch rule of umi_launch applies.  NULL
 * restores the built-in defaults.  Returns UMI_ERR_INVALID_ARG on a
 * malformed table. */
umi_status umi_set_tuning(const char* table_text);

/* Thread-local message for the last non-OK status on this thread. */
const char* umi_last_error(void);

/* Waits for this library's outstanding work and frees every cached
 * workspace.  Call only when no other thread is inside the library. */
void umi_release(void);

/* Library version string. */
const char* umi_version(void);

/* Test hook: the next call on this thread returns `s` without enqueuing
 * anything (UMI_OK disarms it).  Used to exercise error propagation. */
void umi_debug_inject_error(umi_status s);

#ifdef __cplusplus
}
#endif

#endif /* UMI_H */
