/*
 * hawkes_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of the
 * spatiotemporal Hawkes log-likelihood and its gradient, used to check the GPU
 * library.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load this code; the product path never does.  It shares
 * no code with the HIP library.
 *
 * What is computed (paper Section 2.1, equations "likelihood", "fixed",
 * "varying" and "model"; the compensator follows the closed form given right
 * after the R^2 approximation, which cites Laub et al. Section 3.2):
 *
 *   lambda_n = mu * sum_{m : t_m != t_n} N2(|x_n - x_m|^2 ; tau_x^2) * N1(t_n - t_m ; tau_t^2)
 *            + xi * sum_{m : t_m <  t_n} N2(|x_n - x_m|^2 ; h_m^2) * omega * exp(-omega (t_n - t_m))
 *
 *   with h_m = h0 * s_m (the per-source spatial sd; the paper's model 2 uses
 *   sigma_x / sqrt(D_m), i.e. s_m = D_m^(-1/2)), N2(r^2; v) = exp(-r^2/(2v))/(2 pi v)
 *   the isotropic bivariate normal density and N1(d; v) = exp(-d^2/(2v))/sqrt(2 pi v).
 *
 *   Lambda_n = mu * [Phi((t_N - t_n)/tau_t) - Phi(-t_n/tau_t)]
 *            + xi * [1 - exp(-omega (t_N - t_n))],   t_N = max_n t_n, domain (0, t_N]
 *
 *   l_n = log(max(lambda_n, 1e-40)) - Lambda_n     (the floor of Section 2.3.1)
 *   l   = sum_n l_n
 *
 * The background carries the spatial Gaussian N2(.; tau_x^2) (six parameters
 * theta = (mu, tau_x, tau_t, xi, h0, omega)), or, when a spatial-domain area
 * A > 0 is given, the spatially uniform density 1/A of the paper's own models
 * (equation "fixed": mu0 / A(X) times the temporal Gaussian; tau_x then plays
 * no part and its derivative is 0); self pairs and exact time ties
 * are excluded from both sums, as the indicator in equation "fixed" and the
 * appendix kernel's time tests do.  Gradients are the term-by-term partial
 * derivatives of the definition above with respect to theta; a floored event
 * (lambda_n < 1e-40) contributes no gradient from its log term.
 *
 * Per-target sums use Neumaier compensation; the total is summed over rows in
 * index order.  OpenMP parallelises over target rows only, so results do not
 * depend on the thread count.
 *
 * The second half of the file is the Philox4x64-10 counter-based generator
 * (Salmon, Moraes, Dror, Shaw, SC'11) and the uniform within-county location
 * draw of the cut-posterior X-update (paper Section 2.2).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define ORACLE_LAMBDA_FLOOR 1e-40

typedef struct {
    double sum;
    double comp;
} neumaier_t;

static void nm_add(neumaier_t *a, double v)
{
    double t = a->sum + v;
    if (fabs(a->sum) >= fabs(v))
        a->comp += (a->sum - t) + v;
    else
        a->comp += (v - t) + a->sum;
    a->sum = t;
}

static double nm_value(const neumaier_t *a) { return a->sum + a->comp; }

static double std_normal_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

static double std_normal_pdf(double z) { return exp(-0.5 * z * z) / sqrt(2.0 * M_PI); }

/* Isotropic bivariate normal density at squared distance r2 with variance v. */
static double n2_density(double r2, double v) { return exp(-r2 / (2.0 * v)) / (2.0 * M_PI * v); }

/* Univariate normal density at offset d with variance v. */
static double n1_density(double d, double v) { return exp(-d * d / (2.0 * v)) / sqrt(2.0 * M_PI * v); }

enum { P_MU = 0, P_TAUX = 1, P_TAUT = 2, P_XI = 3, P_H0 = 4, P_OMEGA = 5 };

/*
 * For target n: lambda_n and its six partial derivatives d lambda_n / d theta.
 * out[0] = lambda_n, out[1 + k] = d lambda_n / d theta_k.
 */
static void oracle_rate(int64_t nt, int64_t n, const double *t, const double *x, const double *y,
                        const double *s, const double *th, double area, double *out)
{
    const double mu = th[P_MU], taux = th[P_TAUX], taut = th[P_TAUT];
    const double xi = th[P_XI], h0 = th[P_H0], omega = th[P_OMEGA];
    neumaier_t acc[7] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
    const double tn = t[nt], xn = x[nt], yn = y[nt];
    for (int64_t m = 0; m < n; ++m) {
        if (t[m] == tn)
            continue; /* self pair and exact ties: excluded from both sums */
        const double dt = tn - t[m];
        const double dx = xn - x[m], dy = yn - y[m];
        const double d2 = dx * dx + dy * dy;

        /* background pair term and its derivatives */
        if (area > 0.0) {
            /* spatially uniform background: 1/A times the temporal Gaussian */
            const double beta = n1_density(dt, taut * taut) / area;
            nm_add(&acc[0], mu * beta);
            nm_add(&acc[1 + P_MU], beta);
            nm_add(&acc[1 + P_TAUT], mu * beta * (dt * dt / (taut * taut * taut) - 1.0 / taut));
        } else {
        const double beta = n2_density(d2, taux * taux) * n1_density(dt, taut * taut);
        nm_add(&acc[0], mu * beta);
        nm_add(&acc[1 + P_MU], beta);
        nm_add(&acc[1 + P_TAUX], mu * beta * (d2 / (taux * taux * taux) - 2.0 / taux));
        nm_add(&acc[1 + P_TAUT], mu * beta * (dt * dt / (taut * taut * taut) - 1.0 / taut));
        }

        if (t[m] < tn) {
            /* triggering pair term: source m's spatial sd is h0 * s_m */
            const double h = h0 * s[m];
            const double gamma = n2_density(d2, h * h) * omega * exp(-omega * dt);
            nm_add(&acc[0], xi * gamma);
            nm_add(&acc[1 + P_XI], gamma);
            nm_add(&acc[1 + P_H0], xi * gamma * (d2 / (h * h * h0) - 2.0 / h0));
            nm_add(&acc[1 + P_OMEGA], xi * gamma * (1.0 / omega - dt));
        }
    }
    for (int k = 0; k < 7; ++k)
        out[k] = nm_value(&acc[k]);
}

/* Compensator term of event m and its derivatives: out[0] = Lambda_m, out[1+k] = d/d theta_k. */
static void oracle_compensator(double tm, double tN, const double *th, double *out)
{
    const double mu = th[P_MU], taut = th[P_TAUT], xi = th[P_XI], omega = th[P_OMEGA];
    const double a = tN - tm;
    const double bg = std_normal_cdf(a / taut) - std_normal_cdf(-tm / taut);
    const double ea = exp(-omega * a);
    out[0] = mu * bg + xi * (1.0 - ea);
    out[1 + P_MU] = bg;
    out[1 + P_TAUX] = 0.0;
    out[1 + P_TAUT] = -(mu / (taut * taut)) * (a * std_normal_pdf(a / taut) + tm * std_normal_pdf(tm / taut));
    out[1 + P_XI] = 1.0 - ea;
    out[1 + P_H0] = 0.0;
    out[1 + P_OMEGA] = xi * a * ea;
}

/*
 * Log-likelihood restricted to target rows [row_begin, row_end) (the paper's
 * per-GPU slice, Section 2.3.2), its gradient, and optional per-row outputs.
 *
 *   n            number of events (>= 1); t need not be sorted
 *   t, x, y, s   host arrays of length n (days, km, km, bandwidth scale > 0)
 *   theta        (mu, tau_x, tau_t, xi, h0, omega), all > 0
 *   area         0: Gaussian spatial background; > 0: uniform background 1/area (km^2)
 *   loglik       out: sum of l_n over the rows
 *   grad         out (6) or NULL: gradient of that sum with respect to theta
 *   lam, comp    out (row_end - row_begin) or NULL: lambda_n and Lambda_n
 *   ell          out (row_end - row_begin) or NULL: l_n
 *
 * Returns 0, or -1 on invalid arguments.
 */
int hawkes_oracle_loglik(int64_t n, const double *t, const double *x, const double *y, const double *s,
                         const double *theta, double area, int64_t row_begin, int64_t row_end,
                         double *loglik, double *grad, double *lam, double *comp, double *ell)
{
    if (n < 1 || !t || !x || !y || !s || !theta || !loglik || !(area >= 0.0) || !isfinite(area))
        return -1;
    if (row_begin < 0 || row_end > n || row_begin > row_end)
        return -1;
    for (int k = 0; k < 6; ++k)
        if (!(theta[k] > 0.0) || !isfinite(theta[k]))
            return -1;

    double tN = t[0];
    for (int64_t m = 1; m < n; ++m)
        if (t[m] > tN)
            tN = t[m];

    const int64_t rows = row_end - row_begin;
    /* per-row results: l_n and the 6 gradient terms, summed in row order afterwards */
    double *buf = NULL;
    if (rows > 0) {
        buf = (double *)malloc((size_t)rows * 7 * sizeof(double));
        if (!buf)
            return -1;
    }

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < rows; ++r) {
        const int64_t i = row_begin + r;
        double rate[7], cmp[7];
        oracle_rate(i, n, t, x, y, s, theta, area, rate);
        oracle_compensator(t[i], tN, theta, cmp);
        const double lam_i = rate[0];
        const int floored = lam_i < ORACLE_LAMBDA_FLOOR;
        const double l_i = log(floored ? ORACLE_LAMBDA_FLOOR : lam_i) - cmp[0];
        buf[r * 7 + 0] = l_i;
        for (int k = 0; k < 6; ++k)
            buf[r * 7 + 1 + k] = (floored ? 0.0 : rate[1 + k] / lam_i) - cmp[1 + k];
        if (lam)
            lam[r] = lam_i;
        if (comp)
            comp[r] = cmp[0];
        if (ell)
            ell[r] = l_i;
    }

    neumaier_t tot[7] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int64_t r = 0; r < rows; ++r)
        for (int k = 0; k < 7; ++k)
            nm_add(&tot[k], buf[r * 7 + k]);
    free(buf);
    *loglik = nm_value(&tot[0]);
    if (grad)
        for (int k = 0; k < 6; ++k)
            grad[k] = nm_value(&tot[1 + k]);
    return 0;
}

/*
 * The background-only and triggering-only parts of lambda_n for rows
 * [row_begin, row_end): bg[r] = sum over background pair terms (without mu),
 * tr[r] = sum over triggering pair terms (without xi).  Used by the tests that
 * pin each part against an independent computation.
 */
int hawkes_oracle_rate_parts(int64_t n, const double *t, const double *x, const double *y,
                             const double *s, const double *theta, double area, int64_t row_begin,
                             int64_t row_end, double *bg, double *tr)
{
    if (n < 1 || row_begin < 0 || row_end > n || row_begin > row_end || !bg || !tr)
        return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < row_end - row_begin; ++r) {
        double rate[7];
        oracle_rate(row_begin + r, n, t, x, y, s, theta, area, rate);
        bg[r] = rate[1 + P_MU];
        tr[r] = rate[1 + P_XI];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3", */
/* SC'11): 10 rounds of the 4x64 S-box with the published round multipliers   */
/* and Weyl key increments.                                                    */
/* ------------------------------------------------------------------------ */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void hawkes_oracle_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, &hi0, &lo0);
        mulhilo64(M1, c2, &hi1, &lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/*
 * The X-update of the cut posterior (paper Section 2.2): each latent location
 * is drawn uniformly inside its county, here an axis-aligned rectangle
 * rect[c] = (x0, y0, x1, y1).  Event n uses Philox4x64-10 with counter
 * (n, iteration, 0, 0) and key (seed, 0); output words 0 and 1 give
 * u = (w >> 11) * 2^-53 in [0, 1) for x and y, and x = fma(u, x1 - x0, x0).
 */
int hawkes_oracle_resample(int64_t n, const int32_t *county, const double *rect, int32_t n_counties,
                           uint64_t seed, uint64_t iteration, double *x, double *y)
{
    if (n < 0 || (n > 0 && (!county || !rect || !x || !y)) || n_counties < 1)
        return -1;
    for (int64_t i = 0; i < n; ++i)
        if (county[i] < 0 || county[i] >= n_counties)
            return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t ctr[4] = {(uint64_t)i, iteration, 0, 0};
        const uint64_t key[2] = {seed, 0};
        uint64_t w[4];
        hawkes_oracle_philox4x64_10(ctr, key, w);
        const double ux = (double)(w[0] >> 11) * 0x1.0p-53;
        const double uy = (double)(w[1] >> 11) * 0x1.0p-53;
        const double *r = rect + 4 * (int64_t)county[i];
        x[i] = fma(ux, r[2] - r[0], r[0]);
        y[i] = fma(uy, r[3] - r[1], r[1]);
    }
    return 0;
}
