/* sanitize_oracle.c -- driver of the ASan/UBSan build of the FP64 oracle (test infrastructure):
 * runs the oracle's entry points on small event sets, row ranges, the uniform background, the
 * Philox draw and every invalid-argument path, and prints the results for the calling test to
 * compare with the regular build.  Any sanitizer report makes the process fail. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int hawkes_oracle_loglik(int64_t n, const double *t, const double *x, const double *y, const double *s,
                         const double *theta, double area, int64_t row_begin, int64_t row_end, double *loglik,
                         double *grad, double *lam, double *comp, double *ell);
int hawkes_oracle_rate_parts(int64_t n, const double *t, const double *x, const double *y, const double *s,
                             const double *theta, double area, int64_t row_begin, int64_t row_end, double *bg,
                             double *tr);
void hawkes_oracle_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]);
int hawkes_oracle_resample(int64_t n, const int32_t *county, const double *rect, int32_t n_counties, uint64_t seed,
                           uint64_t iteration, double *x, double *y);

static double lcg(uint64_t *st)
{
    *st = *st * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*st >> 11) * 0x1.0p-53;
}

int main(void)
{
    const double theta[6] = {0.5, 10.0, 7.0, 0.3, 2.0, 0.2};
    const int64_t sizes[] = {1, 2, 3, 17, 64};
    for (int k = 0; k < 5; ++k) {
        const int64_t n = sizes[k];
        double *t = malloc(sizeof(double) * n), *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n);
        double *s = malloc(sizeof(double) * n), *lam = malloc(sizeof(double) * n), *comp = malloc(sizeof(double) * n);
        double *ell = malloc(sizeof(double) * n), *bg = malloc(sizeof(double) * n), *tr = malloc(sizeof(double) * n);
        uint64_t st = 12345 + (uint64_t)n;
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            acc += 3.0 * lcg(&st);
            t[i] = floor(acc);  /* integer days: ties */
            x[i] = 50.0 * lcg(&st);
            y[i] = 50.0 * lcg(&st);
            s[i] = 0.5 + lcg(&st);
        }
        for (int a = 0; a < 2; ++a) {
            const double area = a ? 2500.0 : 0.0;
            double ll, g[6];
            if (hawkes_oracle_loglik(n, t, x, y, s, theta, area, 0, n, &ll, g, lam, comp, ell) != 0)
                return 2;
            printf("n %lld area %g loglik %.17g grad %.17g %.17g %.17g %.17g %.17g %.17g\n", (long long)n, area, ll,
                   g[0], g[1], g[2], g[3], g[4], g[5]);
            double lr, gr[6];
            if (hawkes_oracle_loglik(n, t, x, y, s, theta, area, n / 2, n, &lr, gr, NULL, NULL, NULL) != 0)
                return 3;
            if (hawkes_oracle_rate_parts(n, t, x, y, s, theta, area, 0, n, bg, tr) != 0)
                return 4;
        }
        free(t), free(x), free(y), free(s), free(lam), free(comp), free(ell), free(bg), free(tr);
    }
    /* invalid arguments are refused */
    double one = 1.0, ll, g[6];
    if (hawkes_oracle_loglik(0, &one, &one, &one, &one, theta, 0.0, 0, 0, &ll, g, NULL, NULL, NULL) != -1)
        return 5;
    if (hawkes_oracle_loglik(1, &one, &one, &one, &one, theta, -1.0, 0, 1, &ll, g, NULL, NULL, NULL) != -1)
        return 6;
    if (hawkes_oracle_loglik(1, &one, &one, &one, &one, theta, 0.0, 0, 2, &ll, g, NULL, NULL, NULL) != -1)
        return 7;
    if (hawkes_oracle_rate_parts(1, &one, &one, &one, &one, theta, 0.0, 1, 0, &ll, &ll) != -1)
        return 8;
    /* Philox and the location draw */
    uint64_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    hawkes_oracle_philox4x64_10(ctr, key, out);
    printf("philox %llu %llu %llu %llu\n", (unsigned long long)out[0], (unsigned long long)out[1],
           (unsigned long long)out[2], (unsigned long long)out[3]);
    int32_t county[5] = {0, 1, 2, 1, 0};
    double rect[12] = {0, 0, 1, 1, 1, 0, 2, 1, 0, 1, 1, 2}, rx[5], ry[5];
    if (hawkes_oracle_resample(5, county, rect, 3, 7, 9, rx, ry) != 0)
        return 9;
    printf("resample %.17g %.17g %.17g %.17g\n", rx[0], ry[0], rx[4], ry[4]);
    if (hawkes_oracle_resample(5, county, rect, 0, 7, 9, rx, ry) != -1)
        return 10;
    printf("OK\n");
    return 0;
}
