"""Fisher-BT (Algorithm 1) for the oracle: L9 start (Table 1), Fisher scoring
with the relaxed Armijo backtracking of Eq. (4), the stopping and shift rules
of Section 2.1, and a Nelder-Mead fallback.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings of points the paper leaves open (each also listed in the design notes):
  * the step is the full scoring step phi = I^{-1} grad, halved until the relaxed
    Armijo test l(theta+phi) >= l(theta) + c grad.phi - relax passes;
  * a trial with a non-positive component or a covariance that fails Cholesky
    has l = -inf, so the test fails and phi is halved;
  * each distinct theta whose l is computed is one l call (9 for L9, one per
    Armijo trial); the derivatives at an accepted trial are one grad call; a
    user-given start costs one l call and one grad call;
  * the shift happens before an l call beyond ``max_loglik_calls`` or a grad
    call beyond ``max_grad_calls`` (and, if set, after ``max_iter`` steps);
  * the stopping test ||grad||_2 <= grad_tol is checked at every iterate,
    including the start;
  * L9: the first maximum in table order; a failed candidate counts as -inf;
  * Nelder-Mead: reflection 1, expansion 2, contraction 1/2, shrink 1/2 on
    -l; start simplex theta and theta + 0.05 theta_i e_i; stop when the
    spread of l over the vertices is below nm_ftol or after nm_max_evals
    evaluations; its l calls do not count toward the Fisher-scoring budget.
"""
from __future__ import annotations

import math

import numpy as np

# Table 1: weights (w_lower, w_upper) of each candidate coordinate.
_HALF, _LOW, _HIGH = (0.5, 0.5), (5 / 6, 1 / 6), (1 / 6, 5 / 6)
_L9 = (
    (_HALF, _HALF, _HALF),
    (_HALF, _LOW, _LOW),
    (_HALF, _HIGH, _HIGH),
    (_LOW, _HALF, _LOW),
    (_LOW, _LOW, _HIGH),
    (_LOW, _HIGH, _HALF),
    (_HIGH, _HALF, _HIGH),
    (_HIGH, _LOW, _HALF),
    (_HIGH, _HIGH, _LOW),
)


def l9_design(lo, hi):
    """The nine starting candidates of Table 1 for the cube [lo, hi]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    out = np.empty((9, 3))
    for r, row in enumerate(_L9):
        for c, (wl, wu) in enumerate(row):
            out[r, c] = wl * lo[c] + wu * hi[c]
    return out


class OracleEvaluator:
    """Binds data to the oracle's Algorithms 2 and 3; counts calls."""

    def __init__(self, locs, z):
        from . import NotPositiveDefinite, evaluate, loglik

        self._locs = np.asarray(locs, dtype=np.float64)
        self._z = np.asarray(z, dtype=np.float64)
        self._ll, self._ev, self._npd = loglik, evaluate, NotPositiveDefinite

    def loglik(self, theta):
        """l(theta), or -inf for an invalid or non-positive-definite theta."""
        theta = np.asarray(theta, dtype=np.float64)
        if not np.all(np.isfinite(theta)) or np.any(theta <= 0):
            return -math.inf
        try:
            return self._ll(self._locs, self._z, theta)["loglik"]
        except self._npd:
            return -math.inf

    def evaluate(self, theta):
        r = self._ev(self._locs, self._z, theta)
        return r["loglik"], r["score"], r["fisher"]


def nelder_mead(f, x0, ftol=1e-9, max_evals=500, step=0.05):
    """Minimise f from x0 (standard Nelder-Mead, coefficients 1, 2, 1/2, 1/2).

    Returns (x_best, f_best, n_evals).  The vertices are kept sorted by f with
    a stable sort; the loop stops when f(worst) - f(best) < ftol.
    """
    x0 = np.asarray(x0, dtype=np.float64)
    d = x0.size
    simplex = [x0.copy()]
    for i in range(d):
        v = x0.copy()
        v[i] = v[i] + step * x0[i] if x0[i] != 0 else step
        simplex.append(v)
    fv = [f(v) for v in simplex]
    evals = d + 1
    while True:
        order = sorted(range(d + 1), key=lambda k: fv[k])     # stable
        simplex = [simplex[k] for k in order]
        fv = [fv[k] for k in order]
        if not (fv[-1] - fv[0] >= ftol) or evals >= max_evals:
            # also stops on inf - inf (all vertices invalid)
            break
        centroid = np.mean(simplex[:-1], axis=0)
        worst = simplex[-1]
        xr = centroid + (centroid - worst)
        fr = f(xr)
        evals += 1
        if fv[0] <= fr < fv[-2]:
            simplex[-1], fv[-1] = xr, fr
            continue
        if fr < fv[0]:
            xe = centroid + 2.0 * (xr - centroid)
            fe = f(xe)
            evals += 1
            if fe < fr:
                simplex[-1], fv[-1] = xe, fe
            else:
                simplex[-1], fv[-1] = xr, fr
            continue
        if fr < fv[-1]:
            xc = centroid + 0.5 * (xr - centroid)             # outside contraction
            fc = f(xc)
            evals += 1
            if fc <= fr:
                simplex[-1], fv[-1] = xc, fc
                continue
        else:
            xc = centroid - 0.5 * (centroid - worst)          # inside contraction
            fc = f(xc)
            evals += 1
            if fc < fv[-1]:
                simplex[-1], fv[-1] = xc, fc
                continue
        for k in range(1, d + 1):                             # shrink toward the best
            simplex[k] = simplex[0] + 0.5 * (simplex[k] - simplex[0])
            fv[k] = f(simplex[k])
            evals += 1
    return simplex[0], fv[0], evals


def fisher_bt(ev, lo=(0.01, 0.01, 0.01), hi=(5.0, 5.0, 2.0), theta0=None,
              armijo_c=1e-3, armijo_relax=1e-3, backtrack_rho=0.5, grad_tol=1e-3,
              max_loglik_calls=60, max_grad_calls=20, max_iter=0,
              use_nelder_mead=True, nm_ftol=1e-9, nm_max_evals=500, callback=None):
    """Algorithm 1.  ``ev`` provides loglik(theta) (-inf on failure) and
    evaluate(theta) -> (l, grad, I).  Returns a dict with theta, loglik, score,
    fisher, call counts and flags."""
    n_ll = 0
    n_grad = 0
    # ---- initial value ----
    if theta0 is None:
        cands = l9_design(lo, hi)
        best, best_ll = None, -math.inf
        for c in cands:
            v = ev.loglik(c)
            n_ll += 1
            if v > best_ll:                                   # first maximum wins
                best, best_ll = c, v
        if best is None:
            raise ArithmeticError("every L9 candidate failed")
        theta = best.copy()
    else:
        theta = np.asarray(theta0, dtype=np.float64).copy()
        n_ll += 1
    ll, grad, fisher = ev.evaluate(theta)
    n_grad += 1
    it = 0
    if callback:
        callback(it, theta, ll, grad, fisher)
    converged = False
    nm_start = None
    while True:
        if np.linalg.norm(grad) <= grad_tol:
            converged = True
            break
        if max_iter and it >= max_iter:
            break
        phi = np.linalg.solve(fisher, grad)
        accepted = False
        while n_ll < max_loglik_calls:
            trial = theta + phi
            v = ev.loglik(trial)
            n_ll += 1
            if v >= ll + armijo_c * float(grad @ phi) - armijo_relax:
                accepted = True
                break
            phi = backtrack_rho * phi
        if not accepted:
            break
        if n_grad >= max_grad_calls:
            nm_start = trial          # accepted step, but no grad call left for it
            break
        theta = trial
        ll, grad, fisher = ev.evaluate(theta)
        n_grad += 1
        it += 1
        if callback:
            callback(it, theta, ll, grad, fisher)
    used_nm = False
    if not converged and use_nelder_mead:
        used_nm = True
        start = theta if nm_start is None else nm_start
        xbest, fbest, _ = nelder_mead(lambda x: -ev.loglik(x), start, ftol=nm_ftol,
                                      max_evals=nm_max_evals)
        theta = np.asarray(xbest)
        ll, grad, fisher = ev.evaluate(theta)     # one Fisher computation at the result
    return {"theta": theta, "loglik": ll, "score": grad, "fisher": fisher,
            "n_loglik_calls": n_ll, "n_grad_calls": n_grad, "n_iter": it,
            "converged": converged, "used_nelder_mead": used_nm}
