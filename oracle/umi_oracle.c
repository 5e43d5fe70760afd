/*
 * UMI oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the UMI
 * sliding-window asymmetric robust location estimate (arXiv 2604.06602,
 * Section 2).  It exists so that tests, the smoke check and the benchmark's
 * CPU-baseline leg can check the GPU library against it.  Nothing in the
 * product path may call it, and it shares no code, header, table or constant
 * generator with the GPU library.
 *
 * Method (Section 2):
 *   - window: W samples centred on every position (Section 2, opening text);
 *     W = round(0.5 / cadence) | 1 (same place).
 *   - Phase 1 (Section 2.1): location initialised to the exact sample median.
 *   - Phase 2 (Section 2.2, Eq. 1): upper-RMS scale from points strictly
 *     above the median, s = 0.6745 * sigma_upper.
 *   - Phase 3 (Section 2.3, Eqs. 2-4): asymmetric bisquare iterations,
 *     u = (x - mu) / (c s); u_eff = alpha u for u < 0; w = (1 - u_eff^2)^2
 *     for |u_eff| < 1 else 0; mu <- sum(w x) / sum(w).  Fixed iteration count.
 *   - Gap handling and the minimum segment length scaled to W/3
 *     (Section 4.4; Table 3 lists gap handling as a pipeline stage).
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   R1 window = sample-index window centred on i with half-width h=(W-1)/2,
 *      truncated at the ends of the sample's segment (no reflection, no
 *      "valid-only" shrinking of the output);
 *   R2 invalid samples (non-finite flux or time) are skipped inside a window
 *      and get a NaN output;
 *   R3 a new segment starts where consecutive valid times differ by more than
 *      0.5 day (strictly); with no time array there are no breaks;
 *   R4 a segment with fewer than max(1, floor(W/3)) valid samples is dead: NaN;
 *   R5 the median is the lower median, the element of 0-based rank
 *      floor((n-1)/2), ordered by IEEE-754 totalOrder of the float32 bit
 *      patterns (so -0 < +0);
 *   R6 the upper set is strict and numeric (x > median); if it is empty the
 *      scale is 0 and the estimate is the median;
 *   R7 the scale is computed once and held fixed through the iterations;
 *   R8 if sum(w) == 0 in an iteration the location is left unchanged and the
 *      iterations stop; iters = 0 returns the median;
 *   R9 the constant is exactly 0.6745 as printed.
 *   R15 (scale ablation) the standard MAD, which Sections 1 and 2.2 contrast
 *      with the upper-RMS scale and Section 3.1 compares against it, is the
 *      lower median (rank floor((n-1)/2)) of
 *      |x - m| over the window, used unscaled: at the Gaussian model it
 *      equals 0.6745 sigma, the value the upper-RMS scale is normalised to;
 *   R16 per-curve alpha and c (the use-case settings of Table 4) change
 *      nothing else: each curve is estimated with its own pair;
 *   R17 the normalisation stage (a pipeline stage of Table 3) divides the flux
 *      by the trend: detrended = flux / trend, NaN wherever the trend is NaN;
 *   R19 time windows (the window_length in days of Section 4.2, for irregular
 *      cadence): with a window length L, sample i's window keeps only the
 *      valid samples j of its index window (R1) with |t_j - t_i| <= L/2, the
 *      difference taken in float64; W then bounds the samples a window may
 *      hold.
 *
 * Precision: inputs are float32 (flux) and float64 (time); every arithmetic
 * step is float64; the median is returned as the exact float32 element.
 * Built with plain -O2, no fast-math.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_SCALE_CONST 0.6745 /* Section 2.2, after Eq. 1 */
#define ORACLE_GAP_DAYS 0.5       /* reading R3 */
#define ORACLE_SCALE_UPPER_RMS 0  /* Section 2.2, Eq. 1 (the method) */
#define ORACLE_SCALE_MAD 1        /* the ablation, reading R15 */

/* ------------------------------------------------------------------------ */
/* Window-size rule (Section 2, opening text): W = round(0.5 / dt) | 1.      */

int umi_oracle_window_from_cadence(double cadence_days, double window_days)
{
    if (!(cadence_days > 0.0) || !(window_days > 0.0)) return -1;
    double q = window_days / cadence_days;
    if (!(q < 2.0e9)) return -1;
    long r = lround(q); /* round half away from zero; |1 makes ties moot */
    return (int)(r | 1L);
}

/* ------------------------------------------------------------------------ */
/* Eqs. 2-3: asymmetric bisquare weight of a standardised residual u.        */

double umi_oracle_weight(double u, double alpha)
{
    double u_eff = (u < 0.0) ? alpha * u : u; /* Eq. 2 */
    if (fabs(u_eff) < 1.0) {                  /* Eq. 3 */
        double t = 1.0 - u_eff * u_eff;
        return t * t;
    }
    return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Phase 1 (Section 2.1): exact sample median, reading R5.                   */

static uint32_t total_order_key(float f)
{
    uint32_t b;
    memcpy(&b, &f, sizeof b);
    /* negative values: flip all bits; non-negative: set the sign bit */
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

static float key_to_float(uint32_t k)
{
    uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    memcpy(&f, &b, sizeof f);
    return f;
}

static int cmp_u32(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

/* Sorts the n keys (a library sort serves as the ordering step) and takes
 * the element of rank floor((n-1)/2).  `keys` is caller scratch of n. */
static float median_sorted(const float* x, int n, uint32_t* keys)
{
    for (int i = 0; i < n; ++i) keys[i] = total_order_key(x[i]);
    qsort(keys, (size_t)n, sizeof(uint32_t), cmp_u32);
    return key_to_float(keys[(n - 1) / 2]);
}

float umi_oracle_median(const float* x, int n)
{
    if (n <= 0) return NAN;
    uint32_t* keys = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    if (!keys) return NAN;
    float m = median_sorted(x, n, keys);
    free(keys);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Phase 2 (Section 2.2, Eq. 1): s = 0.6745 * sqrt(sum_{x>m}(x-m)^2 / n+).   */

double umi_oracle_upper_scale(const float* x, int n, double m)
{
    double sum_sq = 0.0;
    long n_plus = 0;
    for (int i = 0; i < n; ++i) {
        double xi = (double)x[i];
        if (xi > m) { /* strictly above, reading R6 */
            double d = xi - m;
            sum_sq += d * d;
            ++n_plus;
        }
    }
    if (n_plus == 0) return 0.0;
    return ORACLE_SCALE_CONST * sqrt(sum_sq / (double)n_plus);
}

/* ------------------------------------------------------------------------ */
/* Scale ablation (reading R15): s = lower median of |x_i - m|.              */

static int cmp_f64(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

double umi_oracle_mad_scale(const float* x, int n, double m)
{
    if (n <= 0) return NAN;
    double* dev = (double*)malloc(sizeof(double) * (size_t)n);
    if (!dev) return NAN;
    for (int i = 0; i < n; ++i) dev[i] = fabs((double)x[i] - m);
    qsort(dev, (size_t)n, sizeof(double), cmp_f64);
    double s = dev[(n - 1) / 2];
    free(dev);
    return s;
}

/* ------------------------------------------------------------------------ */
/* One window: Phases 1-3.  Returns the location estimate (the trend value). */

static double window_estimate(const float* x, int n, double alpha, double c,
                              int iters, int scale_mode, uint32_t* keys,
                              float* median_out, double* scale_out)
{
    float med = median_sorted(x, n, keys);
    double m = (double)med;
    double s = (scale_mode == ORACLE_SCALE_MAD) ? umi_oracle_mad_scale(x, n, m)
                                                : umi_oracle_upper_scale(x, n, m);
    if (median_out) *median_out = med;
    if (scale_out) *scale_out = s;
    double mu = m;
    if (!(s > 0.0)) return mu; /* reading R6 */
    double cs = c * s;
    for (int it = 0; it < iters; ++it) {
        double sw = 0.0, swx = 0.0;
        for (int i = 0; i < n; ++i) {
            double xi = (double)x[i];
            double u = (xi - mu) / cs;             /* standardised residual */
            double w = umi_oracle_weight(u, alpha); /* Eqs. 2-3 */
            sw += w;
            swx += w * xi;
        }
        if (sw == 0.0) break; /* reading R8 */
        mu = swx / sw;        /* Eq. 4 */
    }
    return mu;
}

double umi_oracle_window_ex(const float* x, int n, double alpha, double c,
                            int iters, int scale_mode, float* median_out,
                            double* scale_out)
{
    if (n <= 0) {
        if (median_out) *median_out = NAN;
        if (scale_out) *scale_out = NAN;
        return NAN;
    }
    uint32_t* keys = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    if (!keys) return NAN;
    double r = window_estimate(x, n, alpha, c, iters, scale_mode, keys, median_out,
                               scale_out);
    free(keys);
    return r;
}

double umi_oracle_window(const float* x, int n, double alpha, double c,
                         int iters, float* median_out, double* scale_out)
{
    return umi_oracle_window_ex(x, n, alpha, c, iters, ORACLE_SCALE_UPPER_RMS,
                                median_out, scale_out);
}

/* ------------------------------------------------------------------------ */
/* Segmentation (readings R2-R4).  For every sample j of one curve writes the
 * first and last valid index of its segment, or -1/-1 when the sample is
 * invalid or its segment is dead.  Returns the number of segments found.    */

static int sample_valid(const float* flux, const double* time, int64_t j)
{
    if (!isfinite(flux[j])) return 0;
    if (time && !isfinite(time[j])) return 0;
    return 1;
}

int64_t umi_oracle_segments(const float* flux, const double* time, int64_t n,
                            int W, int64_t* seg_lo, int64_t* seg_hi)
{
    int64_t m_min = W / 3;
    if (m_min < 1) m_min = 1;
    int64_t n_seg = 0;
    int64_t j = 0;
    for (int64_t i = 0; i < n; ++i) seg_lo[i] = seg_hi[i] = -1;
    while (j < n) {
        while (j < n && !sample_valid(flux, time, j)) ++j;
        if (j >= n) break;
        /* a segment starts at valid sample j; extend while no gap break */
        int64_t lo = j, hi = j, count = 1, last = j;
        for (int64_t q = j + 1; q < n; ++q) {
            if (!sample_valid(flux, time, q)) continue;
            if (time && (time[q] - time[last]) > ORACLE_GAP_DAYS) break;
            last = q;
            hi = q;
            ++count;
        }
        ++n_seg;
        if (count >= m_min) {
            for (int64_t q = lo; q <= hi; ++q)
                if (sample_valid(flux, time, q)) {
                    seg_lo[q] = lo;
                    seg_hi[q] = hi;
                }
        }
        j = hi + 1;
    }
    return n_seg;
}

/* ------------------------------------------------------------------------ */
/* Per-position estimate over one curve, given segment bounds.               */

static void estimate_at(const float* flux, const double* time, int64_t i, int W,
                        const int64_t* seg_lo, const int64_t* seg_hi,
                        double alpha, double c, int iters, int scale_mode,
                        double window_days, float* buf, uint32_t* keys,
                        double* trend_out, float* median_out)
{
    if (seg_lo[i] < 0) {
        *trend_out = NAN;
        if (median_out) *median_out = NAN;
        return;
    }
    int64_t h = (W - 1) / 2;
    int64_t a = i - h, b = i + h;
    if (a < seg_lo[i]) a = seg_lo[i];
    if (b > seg_hi[i]) b = seg_hi[i];
    int n = 0;
    for (int64_t q = a; q <= b; ++q) {
        if (!sample_valid(flux, time, q)) continue;
        /* reading R19: a time window keeps samples within half its length */
        if (window_days > 0.0 && !(fabs(time[q] - time[i]) <= 0.5 * window_days)) continue;
        buf[n++] = flux[q];
    }
    float med;
    *trend_out = window_estimate(buf, n, alpha, c, iters, scale_mode, keys, &med, NULL);
    if (median_out) *median_out = med;
}

static int params_ok(int64_t n, int W, double alpha, double c, int iters)
{
    if (n < 0 || W < 1 || (W % 2) == 0) return 0;
    if (!(alpha > 0.0) || !isfinite(alpha)) return 0;
    if (!(c > 0.0) || !isfinite(c)) return 0;
    if (iters < 0) return 0;
    return 1;
}

/* Full curve: trend (FP64) and median (exact float32) at every sample.
 * Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
/* window_days > 0 selects time windows (reading R19; needs `time`), else
 * index windows. */
int umi_oracle_detrend_ex(const float* flux, const double* time, int64_t n,
                          int W, double alpha, double c, int iters,
                          int scale_mode, double window_days, double* trend,
                          float* median)
{
    if (!params_ok(n, W, alpha, c, iters)) return -1;
    if (window_days > 0.0 && !time) return -1;
    if (!(window_days <= 0.0 || isfinite(window_days))) return -1;
    if (scale_mode != ORACLE_SCALE_UPPER_RMS && scale_mode != ORACLE_SCALE_MAD) return -1;
    if (n == 0) return 0;
    int64_t* lo = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* hi = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    float* buf = (float*)malloc(sizeof(float) * (size_t)W);
    uint32_t* keys = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)W);
    int rc = 0;
    if (!lo || !hi || !buf || !keys) {
        rc = -2;
        goto done;
    }
    umi_oracle_segments(flux, time, n, W, lo, hi);
    for (int64_t i = 0; i < n; ++i)
        estimate_at(flux, time, i, W, lo, hi, alpha, c, iters, scale_mode,
                    window_days, buf, keys, &trend[i], median ? &median[i] : NULL);
done:
    free(lo);
    free(hi);
    free(buf);
    free(keys);
    return rc;
}

int umi_oracle_detrend(const float* flux, const double* time, int64_t n, int W,
                       double alpha, double c, int iters, double* trend,
                       float* median)
{
    return umi_oracle_detrend_ex(flux, time, n, W, alpha, c, iters,
                                 ORACLE_SCALE_UPPER_RMS, 0.0, trend, median);
}

/* Only at the listed positions of one curve (segments still come from the
 * whole curve): used to check sampled outputs of large workloads. */
int umi_oracle_detrend_at_ex(const float* flux, const double* time, int64_t n,
                             int W, double alpha, double c, int iters,
                             int scale_mode, double window_days,
                             const int64_t* idx, int64_t n_idx, double* trend,
                             float* median)
{
    if (!params_ok(n, W, alpha, c, iters) || n_idx < 0) return -1;
    if (window_days > 0.0 && !time) return -1;
    if (scale_mode != ORACLE_SCALE_UPPER_RMS && scale_mode != ORACLE_SCALE_MAD) return -1;
    for (int64_t k = 0; k < n_idx; ++k)
        if (idx[k] < 0 || idx[k] >= n) return -1;
    if (n_idx == 0) return 0;
    int64_t* lo = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* hi = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    float* buf = (float*)malloc(sizeof(float) * (size_t)W);
    uint32_t* keys = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)W);
    int rc = 0;
    if (!lo || !hi || !buf || !keys) {
        rc = -2;
        goto done;
    }
    umi_oracle_segments(flux, time, n, W, lo, hi);
    for (int64_t k = 0; k < n_idx; ++k)
        estimate_at(flux, time, idx[k], W, lo, hi, alpha, c, iters, scale_mode,
                    window_days, buf, keys, &trend[k], median ? &median[k] : NULL);
done:
    free(lo);
    free(hi);
    free(buf);
    free(keys);
    return rc;
}

int umi_oracle_detrend_at(const float* flux, const double* time, int64_t n,
                          int W, double alpha, double c, int iters,
                          const int64_t* idx, int64_t n_idx, double* trend,
                          float* median)
{
    return umi_oracle_detrend_at_ex(flux, time, n, W, alpha, c, iters,
                                    ORACLE_SCALE_UPPER_RMS, 0.0, idx, n_idx,
                                    trend, median);
}

/* ------------------------------------------------------------------------ */
/* Packed ragged batch: curve b occupies [off_b, off_b + lengths[b]) with off
 * the exclusive prefix sum of lengths.  Curves are shared out over n_threads
 * POSIX threads (each curve is independent).                                */

typedef struct {
    const float* flux;
    const double* time;
    const int64_t* lengths;
    const int64_t* offsets;
    const int* W;
    int64_t n_curves;
    const double* alpha; /* per curve (reading R16) */
    const double* c;
    const double* window_days; /* per curve, or NULL (reading R19) */
    int iters;
    int scale_mode;
    double* trend;
    float* median;
    int64_t next; /* next curve to take, guarded by mu */
    pthread_mutex_t mu;
    int rc;
} batch_job;

static void* batch_worker(void* arg)
{
    batch_job* job = (batch_job*)arg;
    for (;;) {
        pthread_mutex_lock(&job->mu);
        int64_t b = job->next++;
        pthread_mutex_unlock(&job->mu);
        if (b >= job->n_curves) break;
        int64_t off = job->offsets[b];
        int rc = umi_oracle_detrend_ex(
            job->flux + off, job->time ? job->time + off : NULL, job->lengths[b],
            job->W[b], job->alpha[b], job->c[b], job->iters, job->scale_mode,
            job->window_days ? job->window_days[b] : 0.0, job->trend + off,
            job->median ? job->median + off : NULL);
        if (rc != 0) {
            pthread_mutex_lock(&job->mu);
            job->rc = rc;
            pthread_mutex_unlock(&job->mu);
        }
    }
    return NULL;
}

/* Per-curve alpha[b] and c[b] (reading R16) and a scale mode (R15). */
int umi_oracle_detrend_batch_ex(const float* flux, const double* time,
                                const int64_t* lengths, int64_t n_curves,
                                const int* W, const double* alpha,
                                const double* c, const double* window_days,
                                int iters, int scale_mode, double* trend,
                                float* median, int n_threads)
{
    if (n_curves < 0) return -1;
    if (n_curves == 0) return 0;
    int64_t* offsets = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_curves);
    if (!offsets) return -2;
    int64_t acc = 0;
    for (int64_t b = 0; b < n_curves; ++b) {
        if (lengths[b] < 0) {
            free(offsets);
            return -1;
        }
        offsets[b] = acc;
        acc += lengths[b];
    }
    batch_job job = {flux,  time,        lengths, offsets,
                     W,     n_curves,    alpha,   c,
                     window_days, iters, scale_mode, trend,
                     median, 0,          PTHREAD_MUTEX_INITIALIZER, 0};
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t tids[256];
    int started = 0;
    for (int t = 0; t < n_threads; ++t) {
        if (pthread_create(&tids[t], NULL, batch_worker, &job) != 0) break;
        ++started;
    }
    if (started == 0) batch_worker(&job);
    for (int t = 0; t < started; ++t) pthread_join(tids[t], NULL);
    free(offsets);
    return job.rc;
}

int umi_oracle_detrend_batch(const float* flux, const double* time,
                             const int64_t* lengths, int64_t n_curves,
                             const int* W, double alpha, double c, int iters,
                             double* trend, float* median, int n_threads)
{
    if (n_curves < 0) return -1;
    if (n_curves == 0) return 0;
    double* a = (double*)malloc(sizeof(double) * (size_t)n_curves);
    double* cc = (double*)malloc(sizeof(double) * (size_t)n_curves);
    int rc = -2;
    if (a && cc) {
        for (int64_t b = 0; b < n_curves; ++b) {
            a[b] = alpha;
            cc[b] = c;
        }
        rc = umi_oracle_detrend_batch_ex(flux, time, lengths, n_curves, W, a, cc,
                                         NULL, iters, ORACLE_SCALE_UPPER_RMS,
                                         trend, median, n_threads);
    }
    free(a);
    free(cc);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Normalisation (reading R17): detrended[j] = flux[j] / trend[j].           */

void umi_oracle_normalise(const float* flux, const double* trend, int64_t n,
                          double* detrended)
{
    for (int64_t j = 0; j < n; ++j)
        detrended[j] = isnan(trend[j]) ? NAN : (double)flux[j] / trend[j];
}
