/* Sanitizer driver for the FP64 oracle (test infrastructure): random packed
 * batches -- empty, one-sample, gapped, all-invalid and long curves, every
 * odd W up to 2047, both scale estimators, time windows -- through the
 * threaded batch call and the single-position call, built with
 * AddressSanitizer + UndefinedBehaviorSanitizer or ThreadSanitizer.  Prints
 * "oracle checks ok" and exits 0 on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int umi_oracle_detrend_batch_ex(const float* flux, const double* time, const int64_t* lengths,
                                int64_t n_curves, const int* W, const double* alpha,
                                const double* c, const double* window_days, int iters,
                                int scale_mode, double* trend, float* median, int n_threads);
int umi_oracle_detrend_at_ex(const float* flux, const double* time, int64_t n, int W,
                             double alpha, double c, int iters, int scale_mode,
                             double window_days, const int64_t* idx, int64_t n_idx,
                             double* trend, float* median);

static uint64_t s_state = 2604066020ull;
static uint64_t next_u64(void)
{
    s_state ^= s_state << 13;
    s_state ^= s_state >> 7;
    s_state ^= s_state << 17;
    return s_state;
}
static int64_t uni(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1)); }
static double unif(void) { return (double)(next_u64() >> 11) / 9007199254740992.0; }

int main(int argc, char** argv)
{
    int rounds = argc > 1 ? atoi(argv[1]) : 40;
    int failures = 0;
    for (int r = 0; r < rounds; ++r) {
        int64_t n = uni(0, 12);
        int64_t* len = malloc(sizeof(int64_t) * (size_t)(n + 1));
        int* W = malloc(sizeof(int) * (size_t)(n + 1));
        double* a = malloc(sizeof(double) * (size_t)(n + 1));
        double* c = malloc(sizeof(double) * (size_t)(n + 1));
        double* wd = malloc(sizeof(double) * (size_t)(n + 1));
        int64_t total = 0;
        for (int64_t b = 0; b < n; ++b) {
            int kind = (int)uni(0, 5);
            len[b] = kind == 0 ? 0 : (kind == 1 ? 1 : uni(2, 3000));
            W[b] = (int)(uni(0, 1023) * 2 + 1);
            a[b] = 1.0 + 9.0 * unif();
            c[b] = 1.0 + 4.0 * unif();
            wd[b] = uni(0, 2) == 0 ? 0.3 : 0.0;
            total += len[b];
        }
        float* f = malloc(sizeof(float) * (size_t)(total + 1));
        double* t = malloc(sizeof(double) * (size_t)(total + 1));
        double* tr = malloc(sizeof(double) * (size_t)(total + 1));
        float* md = malloc(sizeof(float) * (size_t)(total + 1));
        int64_t o = 0;
        for (int64_t b = 0; b < n; ++b) {
            double tt = 0.0;
            for (int64_t i = 0; i < len[b]; ++i) {
                f[o + i] = (float)(1.0 + 1e-3 * (unif() - 0.5));
                if (uni(0, 30) == 0) f[o + i] = NAN;
                if (uni(0, 500) == 0) tt += 1.0; /* a segment break */
                tt += 2.0 / 1440.0;
                t[o + i] = tt;
            }
            o += len[b];
        }
        int scale = (int)uni(0, 1);
        int rc = umi_oracle_detrend_batch_ex(f, t, len, n, W, a, c, uni(0, 1) ? wd : NULL, 5,
                                             scale, tr, md, (int)uni(1, 8));
        if (rc != 0) {
            fprintf(stderr, "batch rc %d\n", rc);
            ++failures;
        }
        if (n > 0 && len[0] > 0) {
            int64_t idx[3] = {0, len[0] / 2, len[0] - 1};
            double tr3[3];
            float md3[3];
            rc = umi_oracle_detrend_at_ex(f, t, len[0], W[0], a[0], c[0], 5, scale, 0.0, idx, 3,
                                          tr3, md3);
            if (rc != 0) {
                fprintf(stderr, "at rc %d\n", rc);
                ++failures;
            }
        }
        free(len); free(W); free(a); free(c); free(wd); free(f); free(t); free(tr); free(md);
    }
    if (failures) {
        fprintf(stderr, "%d oracle checks failed\n", failures);
        return 1;
    }
    printf("oracle checks ok\n");
    return 0;
}
