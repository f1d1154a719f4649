/*
 * matern_oracle.c -- plain FP64 reference for the Matern covariance and its
 * parameter derivatives (Hong, Abdulah, Genton & Sun, "Fisher Scoring for
 * Exact Matern Covariance Estimation through Stable Smoothness Optimization",
 * Section 2.1 (covariance C(h; theta)) and Section 2.2 (d/d alpha, d/d nu)).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the CPU oracle that the HIP path is
 * checked against.  It shares no code, header, table or constant generator
 * with the product library; only tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.
 *
 * Method (chosen to be slow and obviously correct, not fast):
 *   K_mu(x)        = int_0^inf exp(-x cosh t) cosh(mu t) dt          (DLMF 10.32.9)
 *   dK_mu(x)/dmu   = int_0^inf exp(-x cosh t) t sinh(mu t) dt        (mu-derivative of 10.32.9)
 * evaluated by the trapezoid rule on [0, inf) with step h = min(0.1, 0.45/sqrt(x)),
 * on the exponentially scaled integrand exp(-x (cosh t - 1)) so nothing
 * underflows; cosh t - 1 is formed as 2 sinh^2(t/2).  The sum runs until the
 * integrand is decreasing and its term falls below 1e-18 of the running sum.
 * The trapezoid rule converges geometrically for this analytic, rapidly
 * decaying integrand; the step rule was checked against 40-digit references.
 *
 * Matern entries, with x = h / alpha and c_nu = 2^(1-nu) / Gamma(nu):
 *   C       = sigma2 c_nu x^nu K_nu(x)                                 (Section 2.1)
 *   C_alpha = (sigma2/alpha) c_nu x^(nu+1) K_{nu-1}(x)                 (Section 2.2)
 *   C_nu    = sigma2 c_nu x^nu [ (log(x/2) - psi(nu)) K_nu(x) + dK_nu/dnu ]
 * The last line is the exact nu-derivative of C: the derivative of c_nu is
 * -(log 2 + psi(nu)) c_nu, and d/dnu x^nu = log(x) x^nu.  At h = 0 the
 * covariance is sigma2 for every (alpha, nu), so both derivatives vanish there
 * (the zero-distance case of Supplement A).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

/* Digamma psi(v), v > 0: shift up with psi(v) = psi(v+1) - 1/v until v >= 10,
 * then the asymptotic series psi(v) ~ log v - 1/(2v) - sum B_2k / (2k v^2k)
 * (Abramowitz & Stegun 6.3.18) with Bernoulli numbers B_2..B_14. */
double oracle_digamma(double v)
{
    double acc = 0.0;
    while (v < 10.0) {
        acc -= 1.0 / v;
        v += 1.0;
    }
    double r = 1.0 / (v * v);
    /* B2/2 = 1/12, B4/4 = -1/120, B6/6 = 1/252, B8/8 = -1/240,
       B10/10 = 1/132, B12/12 = -691/32760, B14/14 = 1/12 */
    double series = r * (1.0 / 12 - r * (1.0 / 120 - r * (1.0 / 252 - r * (1.0 / 240
                  - r * (1.0 / 132 - r * (691.0 / 32760 - r * (1.0 / 12)))))));
    return acc + log(v) - 0.5 / v - series;
}

/* Trapezoid sums of the scaled integrals.  kind 0: e^x K_mu(x); kind 1:
 * e^x dK_mu(x)/dmu.  x must be > 0. */
static double scaled_integral(double mu, double x, int kind)
{
    double h = 0.45 / sqrt(x);
    if (h > 0.1)
        h = 0.1;
    double sum = (kind == 0) ? 0.5 : 0.0; /* f(0)/2: cosh(0) = 1, 0*sinh(0) = 0 */
    double amu = fabs(mu);
    for (long j = 1;; ++j) {
        double t = (double)j * h;
        double s = sinh(0.5 * t);
        double e = exp(-x * 2.0 * s * s);
        double f = (kind == 0) ? e * cosh(mu * t) : e * t * sinh(mu * t);
        sum += f;
        /* stop once past the peak of the integrand and negligible */
        if (t > 1.0 && x * sinh(t) > amu + 1.0 && fabs(f) <= 1e-18 * fabs(sum))
            break;
        if (j > 100000000L) /* unreachable for x > 0; guards a NaN input */
            break;
    }
    return h * sum;
}

double oracle_bessel_k_scaled(double mu, double x) { return scaled_integral(mu, x, 0); }
double oracle_bessel_dk_scaled(double mu, double x) { return scaled_integral(mu, x, 1); }

/* The entries selected by `want` (bit 0: C, bit 1: C_alpha, bit 2: C_nu) at
 * distance h >= 0; only the integrals those entries need are evaluated, and
 * the others are left as 0. */
static void matern_entry_sel(double h, double sigma2, double alpha, double nu, int want,
                             double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    if (h == 0.0) {
        out[0] = sigma2;
        return;
    }
    double x = h / alpha;
    double cnu = exp((1.0 - nu) * log(2.0) - lgamma(nu));
    double xnu_emx = exp(nu * log(x) - x); /* x^nu e^{-x}; the K sums carry e^{+x} */
    double k_nu = (want & 5) ? oracle_bessel_k_scaled(nu, x) : 0.0;
    if (want & 1)
        out[0] = sigma2 * cnu * xnu_emx * k_nu;
    if (want & 2) {
        double k_num1 = oracle_bessel_k_scaled(nu - 1.0, x);
        out[1] = (sigma2 / alpha) * cnu * x * xnu_emx * k_num1;
    }
    if (want & 4) {
        double dk_nu = oracle_bessel_dk_scaled(nu, x);
        out[2] = sigma2 * cnu * xnu_emx * ((log(0.5 * x) - oracle_digamma(nu)) * k_nu + dk_nu);
    }
}

/* C, C_alpha, C_nu at distance h >= 0 for theta = (sigma2, alpha, nu). */
void oracle_matern_entry(double h, double sigma2, double alpha, double nu, double out[3])
{
    matern_entry_sel(h, sigma2, alpha, nu, 7, out);
}

/* Entry-wise over a list of distances (used by the pins). */
void oracle_matern_entries(int64_t m, const double *h, double sigma2, double alpha, double nu,
                           double *c, double *c_alpha, double *c_nu)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        double o[3];
        oracle_matern_entry(h[i], sigma2, alpha, nu, o);
        c[i] = o[0];
        c_alpha[i] = o[1];
        c_nu[i] = o[2];
    }
}

/* Full n x n row-major matrices Sigma, Sigma_alpha, Sigma_nu from locations
 * (n x 2, row-major).  Each symmetric pair is evaluated once and mirrored.
 * Any of the output pointers may be NULL. */
void oracle_cov_matrices(int64_t n, const double *locs, double sigma2, double alpha, double nu,
                         double *S, double *Sa, double *Sn)
{
    const int want = (S ? 1 : 0) | (Sa ? 2 : 0) | (Sn ? 4 : 0);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j <= i; ++j) {
            double dx = locs[2 * i] - locs[2 * j];
            double dy = locs[2 * i + 1] - locs[2 * j + 1];
            double o[3];
            matern_entry_sel(sqrt(dx * dx + dy * dy), sigma2, alpha, nu, want, o);
            if (S) {
                S[i * n + j] = o[0];
                S[j * n + i] = o[0];
            }
            if (Sa) {
                Sa[i * n + j] = o[1];
                Sa[j * n + i] = o[1];
            }
            if (Sn) {
                Sn[i * n + j] = o[2];
                Sn[j * n + i] = o[2];
            }
        }
    }
}
