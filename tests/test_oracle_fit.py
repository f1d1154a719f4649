"""Pins of the oracle's Fisher-BT driver (Algorithm 1, Table 1, Eq. (4) and
the stopping/shift rules of Section 2.1)."""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.optimize

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_l9.json")


def test_table1_golden(oracle_mod):
    g = json.load(open(GOLDEN))
    lo, hi = g["simulation_bounds"]["lower"], g["simulation_bounds"]["upper"]
    want = np.array([[g["levels"][c][0] * lo[k] + g["levels"][c][1] * hi[k]
                      for k, c in enumerate(row)] for row in g["rows"]])
    np.testing.assert_allclose(oracle_mod.l9_design(lo, hi), want, rtol=1e-15)
    np.testing.assert_allclose(oracle_mod.l9_design(lo, hi)[0], g["candidate_1_at_simulation_bounds"],
                               rtol=1e-15)


def test_l9_is_an_orthogonal_array(oracle_mod):
    """Every pair of columns of Table 1 shows each pair of levels once."""
    lo, hi = np.zeros(3), np.ones(3)
    D = np.round(oracle_mod.l9_design(lo, hi) * 6).astype(int)   # levels 1, 3, 5
    for a, b in itertools.combinations(range(3), 2):
        assert len(set(zip(D[:, a], D[:, b]))) == 9
    for c in range(3):
        assert sorted(np.bincount(D[:, c]).tolist()) == [0] * 3 + [3, 3, 3]


class Quadratic:
    """l(theta) = -1/2 (theta - m)^T H (theta - m); I = H (exact scoring)."""

    def __init__(self, m, H, fisher_scale=1.0, valid=None):
        self.m, self.H, self.k = np.asarray(m, float), np.asarray(H, float), fisher_scale
        self.valid = valid or (lambda t: True)
        self.nll = self.ngrad = 0

    def loglik(self, t):
        self.nll += 1
        t = np.asarray(t, float)
        if not self.valid(t):
            return -math.inf
        d = t - self.m
        return -0.5 * d @ self.H @ d

    def evaluate(self, t):
        self.ngrad += 1
        d = np.asarray(t, float) - self.m
        return -0.5 * d @ self.H @ d, -self.H @ d, self.k * self.H


H = np.array([[2.0, 0.3, 0.1], [0.3, 1.0, 0.2], [0.1, 0.2, 0.5]])


def test_exact_scoring_converges_in_one_step(oracle_mod):
    ev = Quadratic([1.0, 0.5, 0.7], H)
    r = oracle_mod.fisher_bt(ev, theta0=[3.0, 2.0, 1.5])
    np.testing.assert_allclose(r["theta"], [1.0, 0.5, 0.7], atol=1e-14)
    assert r["converged"] and not r["used_nelder_mead"]
    assert (r["n_loglik_calls"], r["n_grad_calls"], r["n_iter"]) == (2, 2, 1)


def test_armijo_halving(oracle_mod):
    # An information matrix 1/3 of the true curvature makes phi = 3 d (d = theta* - theta).
    # theta + 3d has l = -2 d'Hd and fails Eq. (4); one halving gives theta + 1.5 d
    # (l = -d'Hd / 8), which passes.
    m, t0 = np.array([1.0, 0.5, 0.7]), np.array([1.3, 0.6, 0.8])
    ev = Quadratic(m, H, fisher_scale=1 / 3)
    r = oracle_mod.fisher_bt(ev, theta0=t0, max_iter=1, use_nelder_mead=False)
    np.testing.assert_allclose(r["theta"], t0 + 1.5 * (m - t0), rtol=1e-14)
    assert (r["n_loglik_calls"], r["n_grad_calls"], r["n_iter"]) == (3, 2, 1)


def test_relaxed_armijo_accepts_mirror_step(oracle_mod):
    # With phi = 8 d, two halvings reach theta + 2 d, the mirror image of theta
    # about theta*: equal l, so Eq. (4) with its -0.001 slack accepts it when
    # c grad.phi = 0.002 d'Hd < 0.001.  The iterates then alternate and the
    # gradient budget ends the scoring phase.
    ev = Quadratic([1.0, 0.5, 0.7], H, fisher_scale=1 / 8)
    r = oracle_mod.fisher_bt(ev, theta0=[1.3, 0.6, 0.8], use_nelder_mead=False)
    assert not r["converged"] and r["n_grad_calls"] == 20


def test_invalid_trial_is_minus_infinity(oracle_mod):
    # phi = 3 d: theta + 3d and theta + 1.5d have sigma2 <= 0 (l = -inf), theta + 0.75d passes
    m, t0 = np.array([0.2, 0.5, 0.7]), np.array([0.6, 0.6, 0.8])
    ev = Quadratic(m, H, fisher_scale=1 / 3, valid=lambda t: np.all(t > 0))
    r = oracle_mod.fisher_bt(ev, theta0=t0, max_iter=1, use_nelder_mead=False)
    np.testing.assert_allclose(r["theta"], t0 + 0.75 * (m - t0), rtol=1e-14)
    assert r["n_loglik_calls"] == 4


def test_budget_shift_to_nelder_mead(oracle_mod):
    # a 1000x too large information matrix gives tiny steps: the gradient
    # budget runs out and Nelder-Mead finishes the job
    ev = Quadratic([1.0, 0.5, 0.7], H, fisher_scale=1000.0)
    r = oracle_mod.fisher_bt(ev, theta0=[1.5, 0.9, 1.1])
    assert r["used_nelder_mead"] and r["n_grad_calls"] == 20
    np.testing.assert_allclose(r["theta"], [1.0, 0.5, 0.7], atol=2e-4)
    # no fallback: report the last scoring iterate unconverged
    r2 = oracle_mod.fisher_bt(Quadratic([1.0, 0.5, 0.7], H, fisher_scale=1000.0),
                              theta0=[1.5, 0.9, 1.1], use_nelder_mead=False)
    assert not r2["converged"] and not r2["used_nelder_mead"]


def test_loglik_budget(oracle_mod):
    ev = Quadratic([1.0, 0.5, 0.7], H, fisher_scale=1e-6)   # huge steps: always halving
    r = oracle_mod.fisher_bt(ev, theta0=[1.5, 0.9, 1.1], use_nelder_mead=False)
    assert r["n_loglik_calls"] == 60 and not r["converged"]


def test_l9_start_picks_first_maximum(oracle_mod):
    ev = Quadratic([2.505, 2.505, 1.005], H)
    r = oracle_mod.fisher_bt(ev, lo=(0.01, 0.01, 0.01), hi=(5, 5, 2))
    assert r["n_loglik_calls"] == 9 and r["n_iter"] == 0 and r["converged"]
    np.testing.assert_allclose(r["theta"], [2.505, 2.505, 1.005])


def test_nelder_mead_quadratic(oracle_mod):
    f = lambda x: float((x - [0.3, 2.0, 1.0]) @ H @ (x - [0.3, 2.0, 1.0]))
    x, fx, ne = oracle_mod.nelder_mead(f, np.array([1.0, 1.0, 1.0]), ftol=1e-14, max_evals=2000)
    np.testing.assert_allclose(x, [0.3, 2.0, 1.0], atol=1e-5)
    assert fx < 1e-10 and ne <= 2000


def test_fit_n400_against_scipy(oracle_mod):
    """Fisher-BT from theta0 = (0.5, 0.05, 1.0) on 400 uniform points reaches the
    MLE that a quasi-Newton optimiser finds on the same oracle log-likelihood."""
    w = synth.WORKLOADS["n400"]
    locs, z, _ = synth.dataset(w["n"], w["theta_true"], w["seed"])
    ev = oracle_mod.OracleEvaluator(locs, z)
    r = oracle_mod.fisher_bt(ev, theta0=(0.5, 0.05, 1.0), max_iter=50, grad_tol=1e-8)
    assert r["converged"], r
    assert np.linalg.norm(r["score"]) <= 1e-8
    assert np.all(np.linalg.eigvalsh(r["fisher"]) > 0)
    res = scipy.optimize.minimize(lambda t: -ev.loglik(t), r["theta"] * 1.05,
                                  jac=lambda t: -ev.evaluate(t)[1], method="L-BFGS-B",
                                  bounds=[(1e-6, None)] * 3,
                                  options={"gtol": 1e-10, "ftol": 1e-16, "maxiter": 500})
    np.testing.assert_allclose(r["theta"], res.x, rtol=1e-6)
