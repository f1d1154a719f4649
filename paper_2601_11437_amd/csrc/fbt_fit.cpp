// Fisher-BT driver (Algorithm 1): L9 start (Table 1), Fisher scoring with the
// relaxed Armijo backtracking of Eq. (4), the stopping and shift rules of
// Section 2.1, and a Nelder-Mead fallback.  Host-only; the evaluations come
// from an fbt_evaluator (the GPU one in fbt_fit).
//
// Readings of points the paper leaves open:
//  - step phi = I^{-1} grad (no damping); halving applies to phi itself;
//  - a trial with a component <= 0 or a covariance that is not positive
//    definite has l = -inf, so Eq. (4) fails and phi is halved;
//  - call counting: each theta whose l is computed is one l call (nine for L9,
//    one per Armijo trial); the derivatives at an accepted trial (which reuse
//    its factorisation) are one grad call; a user-given start costs one of each;
//  - shift before an l call beyond max_loglik_calls or a grad call beyond
//    max_grad_calls, or after max_iter accepted steps when max_iter > 0;
//  - the stopping test ||grad||_2 <= grad_tol is checked at every iterate,
//    including the start;
//  - L9: first maximum in table order; failed candidates count as -inf;
//  - Nelder-Mead on -l: coefficients 1, 2, 1/2, 1/2; start simplex theta and
//    theta + 0.05 theta_i e_i; vertices kept in a stable order of -l; stop when
//    the spread of l over the vertices is below nm_ftol or after nm_max_evals
//    evaluations.  Its l calls do not count toward the scoring budget.
#include "fisherbt.h"
#include "fbt_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace {

const double INF = std::numeric_limits<double>::infinity();

bool positive3(const double *t)
{
    return std::isfinite(t[0]) && std::isfinite(t[1]) && std::isfinite(t[2]) && t[0] > 0 &&
           t[1] > 0 && t[2] > 0;
}

// l(theta) or -inf; other errors are returned in *err.
double loglik_or_minus_inf(const fbt_evaluator *ev, const double *t, fbt_status *err)
{
    *err = FBT_OK;
    if (!positive3(t))
        return -INF;
    double v = 0.0;
    fbt_status s = ev->loglik(ev->user, t, &v);
    if (s == FBT_ENOTPD || s == FBT_ENONFINITE)
        return -INF;
    if (s != FBT_OK) {
        *err = s;
        return -INF;
    }
    return std::isfinite(v) ? v : -INF;
}

// Solve the 3x3 system I phi = g by Gaussian elimination with partial pivoting.
bool solve3(const double *I, const double *g, double *phi)
{
    double a[3][4];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            a[i][j] = I[3 * i + j];
        a[i][3] = g[i];
    }
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int r = c + 1; r < 3; ++r)
            if (std::fabs(a[r][c]) > std::fabs(a[p][c]))
                p = r;
        if (!(std::fabs(a[p][c]) > 0.0))
            return false;
        if (p != c)
            for (int j = 0; j < 4; ++j)
                std::swap(a[c][j], a[p][j]);
        for (int r = c + 1; r < 3; ++r) {
            const double f = a[r][c] / a[c][c];
            for (int j = c; j < 4; ++j)
                a[r][j] -= f * a[c][j];
        }
    }
    for (int i = 2; i >= 0; --i) {
        double s = a[i][3];
        for (int j = i + 1; j < 3; ++j)
            s -= a[i][j] * phi[j];
        phi[i] = s / a[i][i];
    }
    return std::isfinite(phi[0]) && std::isfinite(phi[1]) && std::isfinite(phi[2]);
}

double norm3(const double *v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

struct Vertex {
    double x[3];
    double f; // -l
};

// Nelder-Mead minimisation of -l from x0; returns the best vertex.
fbt_status nelder_mead(const fbt_evaluator *ev, const double *x0, double ftol, int max_evals,
                       Vertex *best, int *evals_out)
{
    fbt_status err = FBT_OK;
    Vertex v[4];
    int evals = 0;
    auto f = [&](const double *x) {
        ++evals;
        return -loglik_or_minus_inf(ev, x, &err);
    };
    for (int i = 0; i < 4; ++i) {
        std::memcpy(v[i].x, x0, sizeof(v[i].x));
        if (i > 0)
            v[i].x[i - 1] = (x0[i - 1] != 0.0) ? x0[i - 1] + 0.05 * x0[i - 1] : 0.05;
        v[i].f = f(v[i].x);
        if (err != FBT_OK)
            return err;
    }
    for (;;) {
        std::stable_sort(v, v + 4, [](const Vertex &a, const Vertex &b) { return a.f < b.f; });
        if (!(v[3].f - v[0].f >= ftol) || evals >= max_evals)
            break;
        double c[3], xr[3];
        for (int k = 0; k < 3; ++k) {
            c[k] = ((v[0].x[k] + v[1].x[k]) + v[2].x[k]) / 3.0;
            xr[k] = c[k] + (c[k] - v[3].x[k]);
        }
        const double fr = f(xr);
        if (err != FBT_OK)
            return err;
        if (v[0].f <= fr && fr < v[2].f) {
            std::memcpy(v[3].x, xr, sizeof(xr));
            v[3].f = fr;
            continue;
        }
        if (fr < v[0].f) {
            double xe[3];
            for (int k = 0; k < 3; ++k)
                xe[k] = c[k] + 2.0 * (xr[k] - c[k]);
            const double fe = f(xe);
            if (err != FBT_OK)
                return err;
            if (fe < fr) {
                std::memcpy(v[3].x, xe, sizeof(xe));
                v[3].f = fe;
            } else {
                std::memcpy(v[3].x, xr, sizeof(xr));
                v[3].f = fr;
            }
            continue;
        }
        double xc[3];
        bool accept;
        if (fr < v[3].f) { // outside contraction
            for (int k = 0; k < 3; ++k)
                xc[k] = c[k] + 0.5 * (xr[k] - c[k]);
            const double fc = f(xc);
            if (err != FBT_OK)
                return err;
            accept = fc <= fr;
            if (accept) {
                std::memcpy(v[3].x, xc, sizeof(xc));
                v[3].f = fc;
            }
        } else { // inside contraction
            for (int k = 0; k < 3; ++k)
                xc[k] = c[k] - 0.5 * (c[k] - v[3].x[k]);
            const double fc = f(xc);
            if (err != FBT_OK)
                return err;
            accept = fc < v[3].f;
            if (accept) {
                std::memcpy(v[3].x, xc, sizeof(xc));
                v[3].f = fc;
            }
        }
        if (accept)
            continue;
        for (int i = 1; i < 4; ++i) { // shrink toward the best vertex
            for (int k = 0; k < 3; ++k)
                v[i].x[k] = v[0].x[k] + 0.5 * (v[i].x[k] - v[0].x[k]);
            v[i].f = f(v[i].x);
            if (err != FBT_OK)
                return err;
        }
    }
    *best = v[0];
    *evals_out = evals;
    return FBT_OK;
}

} // namespace

extern "C" {

void fbt_l9_design(const double lo[3], const double hi[3], double out[27])
{
    // Table 1: per candidate and coordinate, the weight on the upper corner
    // (levels 1/2, 1/6, 5/6; the lower corner gets one minus it).
    static const double H = 0.5, L = 1.0 / 6.0, U = 5.0 / 6.0;
    static const double w[9][3] = {{H, H, H}, {H, L, L}, {H, U, U}, {L, H, L}, {L, L, U},
                                   {L, U, H}, {U, H, U}, {U, L, H}, {U, U, L}};
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 3; ++c) {
            const double wu = w[r][c];
            const double wl = (wu == H) ? H : (wu == L ? 5.0 / 6.0 : 1.0 / 6.0);
            out[3 * r + c] = wl * lo[c] + wu * hi[c];
        }
}

void fbt_fit_options_default(fbt_fit_options *o)
{
    if (!o)
        return;
    std::memset(o, 0, sizeof(*o));
    o->theta0 = nullptr;
    o->lo[0] = o->lo[1] = o->lo[2] = 0.01;
    o->hi[0] = 5.0;
    o->hi[1] = 5.0;
    o->hi[2] = 2.0;
    o->armijo_c = 1e-3;
    o->armijo_relax = 1e-3;
    o->backtrack_rho = 0.5;
    o->grad_tol = 1e-3;
    o->max_loglik_calls = 60;
    o->max_grad_calls = 20;
    o->max_iter = 0;
    o->nelder_mead = 1;
    o->nm_ftol = 1e-9;
    o->nm_max_evals = 500;
    o->mixed_switch = 1e-4;
}

fbt_status fbt_fit_evaluator(const fbt_evaluator *ev, const fbt_fit_options *opt,
                             fbt_fit_result *out)
{
    if (!ev || !ev->loglik || !ev->eval || !opt || !out)
        return FBT_EINVAL;
    if (!(opt->backtrack_rho > 0 && opt->backtrack_rho < 1) || opt->max_loglik_calls < 1 ||
        opt->max_grad_calls < 1 || !(opt->grad_tol >= 0) || opt->nm_max_evals < 4)
        return FBT_EINVAL;
    std::memset(out, 0, sizeof(*out));
    out->precision_switch = -1;
    fbt_status err = FBT_OK;
    int n_ll = 0, n_grad = 0, it = 0;
    double theta[3];
    // ---- initial value ----
    if (!opt->theta0) {
        if (!positive3(opt->lo) || !positive3(opt->hi))
            return FBT_EINVAL;
        double cand[27];
        fbt_l9_design(opt->lo, opt->hi, cand);
        int best = -1;
        double best_ll = -INF;
        for (int r = 0; r < 9; ++r) {
            const double v = loglik_or_minus_inf(ev, cand + 3 * r, &err);
            ++n_ll;
            if (err != FBT_OK)
                return err;
            if (v > best_ll) {
                best_ll = v;
                best = r;
            }
        }
        if (best < 0)
            return FBT_ENOTPD;
        std::memcpy(theta, cand + 3 * best, sizeof(theta));
    } else {
        if (!positive3(opt->theta0))
            return FBT_EINVAL;
        std::memcpy(theta, opt->theta0, sizeof(theta));
        ++n_ll;
    }
    double ll, grad[3], fisher[9];
    fbt_status s = ev->eval(ev->user, theta, &ll, grad, fisher);
    ++n_grad;
    if (s != FBT_OK)
        return s;
    if (opt->cb)
        opt->cb(opt->cb_user, it, theta, ll, grad, fisher);
    bool converged = false, have_nm_start = false;
    double nm_start[3];
    for (;;) {
        if (norm3(grad) <= opt->grad_tol) {
            converged = true;
            break;
        }
        if (opt->max_iter > 0 && it >= opt->max_iter)
            break;
        double phi[3];
        if (!solve3(fisher, grad, phi))
            break;
        bool accepted = false;
        double trial[3];
        while (n_ll < opt->max_loglik_calls) {
            for (int k = 0; k < 3; ++k)
                trial[k] = theta[k] + phi[k];
            const double v = loglik_or_minus_inf(ev, trial, &err);
            ++n_ll;
            if (err != FBT_OK)
                return err;
            const double gphi = grad[0] * phi[0] + grad[1] * phi[1] + grad[2] * phi[2];
            if (v >= ll + opt->armijo_c * gphi - opt->armijo_relax) {
                accepted = true;
                break;
            }
            for (int k = 0; k < 3; ++k)
                phi[k] *= opt->backtrack_rho;
        }
        if (!accepted)
            break;
        if (n_grad >= opt->max_grad_calls) {
            std::memcpy(nm_start, trial, sizeof(trial));
            have_nm_start = true;
            break;
        }
        std::memcpy(theta, trial, sizeof(theta));
        s = ev->eval(ev->user, theta, &ll, grad, fisher);
        ++n_grad;
        if (s != FBT_OK)
            return s;
        ++it;
        if (opt->cb)
            opt->cb(opt->cb_user, it, theta, ll, grad, fisher);
    }
    int used_nm = 0, nm_evals = 0;
    if (!converged && opt->nelder_mead) {
        used_nm = 1;
        Vertex best;
        if ((s = nelder_mead(ev, have_nm_start ? nm_start : theta, opt->nm_ftol,
                             opt->nm_max_evals, &best, &nm_evals)) != FBT_OK)
            return s;
        std::memcpy(theta, best.x, sizeof(theta));
        // one Fisher computation at the result
        if ((s = ev->eval(ev->user, theta, &ll, grad, fisher)) != FBT_OK)
            return s;
    }
    std::memcpy(out->theta, theta, sizeof(theta));
    out->loglik = ll;
    std::memcpy(out->score, grad, sizeof(grad));
    std::memcpy(out->fisher, fisher, sizeof(fisher));
    out->n_loglik_calls = n_ll;
    out->n_grad_calls = n_grad;
    out->n_iter = it;
    out->used_nelder_mead = used_nm;
    out->converged = converged ? 1 : 0;
    out->n_nm_evals = nm_evals;
    if (!converged && !opt->nelder_mead)
        return FBT_EBUDGET;
    return FBT_OK;
}

// The GPU evaluator of fbt_fit: derivative evaluations go through
// fbt::fit_eval, which moves a mixed-precision context to FP64 near the
// optimum; the driver itself is unchanged.
struct GpuFit {
    fbt_ctx *ctx;
    int fp64_ctx;      // the context started in FP64
    double sw;         // fbt_fit_options.mixed_switch
    int state;         // 1 once the derivatives run in FP64
    int calls, n_fp64, switch_at;
};

static fbt_status gpu_loglik(void *user, const double theta[3], double *ll)
{
    return fbt_loglik(((GpuFit *)user)->ctx, theta, ll);
}

static fbt_status gpu_eval(void *user, const double theta[3], double *ll, double score[3],
                           double fisher[9])
{
    GpuFit *g = (GpuFit *)user;
    const int before = g->state;
    const fbt_status s = fbt::fit_eval(g->ctx, theta, g->sw, &g->state, ll, score, fisher);
    if (s == FBT_OK) {
        if (g->fp64_ctx || g->state)
            ++g->n_fp64;
        if (!before && g->state)
            g->switch_at = g->calls;
        ++g->calls;
    }
    return s;
}

fbt_status fbt_fit(fbt_ctx *ctx, const fbt_fit_options *opt, fbt_fit_result *out)
{
    if (!ctx || !opt || !(opt->mixed_switch >= 0))
        return FBT_EINVAL;
    const int32_t prec = fbt::ctx_precision(ctx);
    // The line search's acceptance tests (Eq. (4)) take FP64 log-likelihoods;
    // under FBT_MIXED_FP32_ALL and _BF16_ALL fbt_loglik carries the low
    // precision rounding of the factorisation, which no refinement of the
    // solves removes.
    if (prec == FBT_MIXED_FP32_ALL || prec == FBT_MIXED_BF16_ALL)
        return FBT_EINVAL;
    GpuFit g = {ctx, prec == FBT_FP64, opt->mixed_switch, 0, 0, 0, -1};
    fbt_evaluator ev = {&g, gpu_loglik, gpu_eval};
    const fbt_status s = fbt_fit_evaluator(&ev, opt, out);
    fbt_set_precision(ctx, prec);
    if (out && (s == FBT_OK || s == FBT_EBUDGET)) {
        out->n_fp64_evals = g.n_fp64;
        out->precision_switch = g.switch_at;
    }
    return s;
}

} // extern "C"
