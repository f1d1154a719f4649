// Device functions shared by the kernel files: the FP64 MFMA wrapper and the
// Matern entries (covariance and its two derivatives) by quadrature.
#pragma once
#include "fbt_internal.h"

#include <math.h>

namespace fbt {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    // D(16x16) = A(16x4) B(4x16) + C.  Lane l supplies A[l%16][l/16] and
    // B[l/16][l%16]; it holds D[l/16 + 4r][l%16] in element r.
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Covariance generation (Section 2.1; derivatives Section 2.2)
//
// With x = h / alpha and the exponentially scaled integrals
//   SK  = e^x K_nu(x)      = int_0^inf e^{-x (cosh t - 1)} cosh(nu t) dt
//   SK1 = e^x K_{nu-1}(x)  = int_0^inf e^{-x (cosh t - 1)} cosh((nu-1) t) dt
//   SD  = e^x dK_nu/dnu(x) = int_0^inf e^{-x (cosh t - 1)} t sinh(nu t) dt
// (the integral form of K and its order derivative), each entry is
//   C       = sigma2 c_nu E SK,            E = x^nu e^{-x}, c_nu = 2^(1-nu)/Gamma(nu)
//   C_alpha = sigma2/alpha c_nu x E SK1
//   C_nu    = sigma2 c_nu E ((log x - log 2 - psi(nu)) SK + SD)
// The integrals use the trapezoid rule with step h_L = 0.2 / 2^L, where the
// level L is the smallest with x <= 9 * 4^L (so h_L <= 0.6 / sqrt(x)), and
// stop past the t where x (cosh t - 1) - (|nu| + 1) t reaches 45 (an upper
// bound of it): beyond it the integrands are below e^-45 of their value at
// t = 0.  At x = 0 the entry is (sigma2, 0, 0).
// ---------------------------------------------------------------------------

__device__ __forceinline__ double acosh_ge1(double y) { return log(y + sqrt((y - 1.0) * (y + 1.0))); }

// Paper mode (Supplementary A): d/dnu [x^nu K_nu(x)] by the first case that
// applies: (2) x < 8.5, nu not within 1e-6 of an integer: the power series of
// K_nu differentiated term by term (20 terms, coefficients per theta in
// pc[PC_A1 / PC_B0 / PC_B1]); (3) 8.5 <= x < 30: the nu-derivative of the
// uniform expansion of K_nu(nu z), z = x / nu (12 terms below x = 15, 8
// beyond; the three sums are polynomials in p = (1 + z^2)^{-1/2} with
// per-theta coefficients); (4) x >= 30, nu + 1/2 not within 1e-6 of an
// integer: the nu-derivative of the Hankel expansion (5 terms); (5) otherwise
// the central difference with lag 1e-9 of x^nu K_nu(x), whose two values
// come from the quadrature with the cosh((nu +- lag) t) weights (skp, skm).
__device__ __forceinline__ double paper_dxk(const GenParams &gp, double x, double lx, double skp,
                                            double skm)
{
    const double nu = gp.nu;
    const double *pc = gp.pc;
    if (x < 8.5 && !gp.fd_small) {
        const double x2 = 0.25 * x * x, x2nu = exp(2.0 * nu * lx), tl = 2.0 * lx * x2nu;
        double acc = 0.0;
        for (int k = PC_SER - 1; k >= 0; --k)
            acc = fma(acc, x2, fma(tl, pc[PC_B0 + k], fma(x2nu, pc[PC_B1 + k], pc[PC_A1 + k])));
        return acc;
    }
    if (x >= 8.5 && x < 30.0) {
        const double z = x / nu, q = fma(z, z, 1.0), sq = sqrt(q), p = 1.0 / sq;
        const double eta = sq + log(z / (1.0 + sq));
        const double g = exp(nu * (lx - eta)) * pc[PC_SQPI] / sqrt(sq);
        const double *d = pc + (x < 15.0 ? PC_D12 : PC_D8);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int j = PC_DEB - 1; j >= 0; --j) {
            s0 = fma(s0, p, d[j]);
            s1 = fma(s1, p, d[PC_DEB + j]);
            s2 = fma(s2, p, d[2 * PC_DEB + j]);
        }
        const double lead = pc[PC_LOGNU] + log(1.0 + sq) - 0.5 / (nu * q);
        return g * (lead * s0 - s1 + (x * x / (nu * nu * nu)) / (q * sq) * s2);
    }
    if (x >= 30.0 && !gp.fd_large) {
        const double r = 1.0 / x;
        double acc = 0.0;
        for (int k = PC_HAN - 1; k >= 0; --k)
            acc = fma(acc, r, fma(lx, pc[PC_HA + k], pc[PC_HB + k]));
        return 1.2533141373155003 * exp((nu - 0.5) * lx - x) * acc; // sqrt(pi / 2)
    }
    const double fp = exp((nu + PAPER_LAG) * lx - x) * skp;
    const double fm = exp((nu - PAPER_LAG) * lx - x) * skm;
    return (fp - fm) / (2.0 * PAPER_LAG);
}

__device__ __forceinline__ void matern3(const GenParams &gp, const Node *tab, double x, int mode,
                                        double &c, double &ca, double &cn)
{
    if (x == 0.0) {
        c = gp.sigma2;
        ca = 0.0;
        cn = 0.0;
        return;
    }
    if (!(x <= gp.xtop[NLEV - 1])) { // beyond every level: e^{-x} underflows
        c = 0.0;
        ca = 0.0;
        cn = 0.0;
        return;
    }
    int L = 0;
#pragma unroll
    for (int l = 0; l < NLEV - 1; ++l)
        L += (x > gp.xtop[l]);
    // the level's step, first node and node count, selected with constant
    // indices (a copy of gp then stays in registers)
    double h = gp.h[0];
    int lev_len = gp.len[0], lev_off = gp.off[0];
#pragma unroll
    for (int l = 1; l < NLEV; ++l)
        if (L == l) {
            h = gp.h[l];
            lev_len = gp.len[l];
            lev_off = gp.off[l];
        }
    // truncation point: the root t* of F(t) = x (cosh t - 1) - g t - 45.  The
    // iterates t1 = acosh(1 + 45 / x), t2 = acosh(1 + (45 + g t1) / x) rise
    // towards it with F(t2) = -g (t2 - t1), and beyond t2 the slope of F is at
    // least x (cosh t2 - 1) - g = 45 + g t1 - g, so t2 + g (t2 - t1) / (45 - g)
    // bounds t* from above (for g < 45; larger g falls back to the table's end)
    const double g = gp.abs_nu + 1.0;
    const double t1 = acosh_ge1(1.0 + 45.0 / x);
    const double t2 = acosh_ge1(1.0 + (45.0 + g * t1) / x);
    double t = g < 44.0 ? t2 + g * (t2 - t1) / (45.0 - g) : 1.0e4;
    t = fmin(t, 1.0e4); // x below ~1e-300: every node of the level
    int J = (int)(t / h) + 2;
    J = J < lev_len ? J : lev_len;
    const Node *nd = tab + lev_off;
    double sk = 0.0, sk1 = 0.0, sd = 0.0, skp = 0.0, skm = 0.0;
    if (mode == GEN_SIGMA) {
        for (int j = 0; j < J; ++j) {
            const double e = exp(-x * nd[j].cm1);
            sk = fma(e, nd[j].wk, sk);
        }
    } else if (!gp.paper) {
        for (int j = 0; j < J; ++j) {
            const double e = exp(-x * nd[j].cm1);
            sk = fma(e, nd[j].wk, sk);
            sk1 = fma(e, nd[j].wk1, sk1);
            sd = fma(e, nd[j].wd, sd);
        }
    } else {
        for (int j = 0; j < J; ++j) {
            const double e = exp(-x * nd[j].cm1);
            sk = fma(e, nd[j].wk, sk);
            sk1 = fma(e, nd[j].wk1, sk1);
            skp = fma(e, nd[j].wkp, skp);
            skm = fma(e, nd[j].wkm, skm);
        }
    }
    const double lx = log(x);
    const double E = gp.cnu * exp(gp.nu * lx - x); // c_nu x^nu e^{-x}
    c = gp.sigma2 * E * sk;
    ca = gp.sigma2 / gp.alpha * x * E * sk1;
    if (!gp.paper)
        cn = gp.sigma2 * E * ((lx - gp.log2_psi) * sk + sd);
    else
        cn = (mode == GEN_SIGMA) ? 0.0
                                 : gp.sigma2 * gp.cnu *
                                       (paper_dxk(gp, x, lx, skp, skm) -
                                        gp.log2_psi * exp(gp.nu * lx - x) * sk);
}

}  // namespace fbt
