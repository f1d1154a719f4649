"""Pins of the oracle's Algorithms 2 and 3 (log-likelihood Eq. (1), score
Eq. (2), Fisher information Eq. (3), trace identity Eq. (5)).

The references are independent of the oracle's Cholesky/solve route: closed
forms at n = 1 and n = 2, Eqs. (1)-(3) evaluated literally with a 30-digit
explicit inverse and determinant (mpmath), invariances of the model, central
differences of the log-likelihood, and Monte Carlo moments of the score.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import synth


def _data(n, seed, theta=(1.0, 0.1, 0.5)):
    locs, z, _ = synth.dataset(n, theta, seed)
    return locs, z


def test_n1_closed_form(oracle_mod):
    for s2, z in ((1.0, 0.3), (2.5, -1.7), (0.04, 0.01)):
        theta = (s2, 0.2, 1.3)
        r = oracle_mod.evaluate(np.array([[0.3, 0.4]]), np.array([z]), theta)
        ll = -0.5 * math.log(2 * math.pi) - 0.5 * math.log(s2) - z * z / (2 * s2)
        assert abs(r["loglik"] - ll) < 1e-15 * max(1, abs(ll))
        np.testing.assert_allclose(r["score"], [(z * z / s2 - 1) / (2 * s2), 0, 0], atol=1e-15)
        assert r["fisher"][0, 0] == 1 / (2 * s2 ** 2)
        np.testing.assert_array_equal(r["fisher"][1:, :], 0.0)


def test_n2_closed_form(oracle_mod):
    locs = np.array([[0.1, 0.2], [0.25, 0.1]])
    z = np.array([0.7, -0.2])
    h = float(np.hypot(*(locs[0] - locs[1])))
    for theta in ((1.0, 0.1, 0.5), (1.7, 0.3, 2.5)):
        c, _, _ = oracle_mod.matern_entries([h], theta)
        s2, c = theta[0], c[0]
        det = s2 * s2 - c * c
        quad = (s2 * z[0] ** 2 - 2 * c * z[0] * z[1] + s2 * z[1] ** 2) / det
        ll = -math.log(2 * math.pi) - 0.5 * math.log(det) - 0.5 * quad
        assert abs(oracle_mod.loglik(locs, z, theta)["loglik"] - ll) < 1e-14 * abs(ll)


def _brute_force(oracle_mod, locs, z, theta, dps=30):
    """Eqs. (1)-(3) literally, with a 30-digit inverse and determinant."""
    mp.mp.dps = dps
    S, Sa, Sn = oracle_mod.cov_matrices(locs, theta)
    Sg = S / theta[0]                                    # Sigma_{sigma2} = Sigma / sigma2
    n = z.size
    M = mp.matrix(S.tolist())
    Minv = M ** -1
    Zm = mp.matrix(z.tolist())
    ll = -mp.mpf(n) / 2 * mp.log(2 * mp.pi) - mp.log(mp.det(M)) / 2 - (Zm.T * Minv * Zm)[0] / 2
    A = [Minv * mp.matrix(D.tolist()) for D in (Sg, Sa, Sn)]
    w = Minv * Zm
    score = []
    for Di, Ai in zip((Sg, Sa, Sn), A):
        tr = sum(Ai[k, k] for k in range(n))
        q = (w.T * mp.matrix(Di.tolist()) * w)[0]
        score.append(-tr / 2 + q / 2)
    fisher = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            P = A[i] * A[j]
            fisher[i, j] = float(sum(P[k, k] for k in range(n)) / 2)
    return float(ll), np.array([float(s) for s in score]), fisher


@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.5), (0.6, 0.05, 1.4), (2.0, 0.2, 0.25)])
def test_brute_force_small_n(oracle_mod, theta):
    locs, z = _data(20, 11)
    ll, score, fisher = _brute_force(oracle_mod, locs, z, theta)
    r = oracle_mod.evaluate(locs, z, theta)
    assert abs(r["loglik"] - ll) < 1e-12 * abs(ll)
    scale = np.abs(score) + np.abs(np.diag(fisher)) + 1.0
    np.testing.assert_allclose(r["score"], score, rtol=0, atol=1e-11 * scale.max())
    np.testing.assert_allclose(r["fisher"], fisher, rtol=1e-11)


def test_trace_identity_eq5(oracle_mod):
    locs, z = _data(60, 3)
    r = oracle_mod.evaluate(locs, z, (1.2, 0.08, 0.9))
    for k in ("aa", "an", "nn"):
        a, b = r["trAB_frobenius"][k], r["trAB_direct"][k]
        assert abs(a - b) <= 1e-11 * abs(b)
    gen = np.random.default_rng(0)
    A, B = gen.standard_normal((2, 17, 17))
    assert abs(oracle_mod.trace_product_frobenius(A, B) - np.trace(A @ B)) < 1e-12


def test_fisher_structure(oracle_mod):
    locs, z = _data(80, 5)
    for theta in ((1.0, 0.1, 0.5), (0.3, 0.3, 1.8), (4.0, 0.02, 0.1)):
        r = oracle_mod.evaluate(locs, z, theta)
        I = r["fisher"]
        np.testing.assert_array_equal(I, I.T)
        assert I[0, 0] == 80 / (2 * theta[0] ** 2)
        assert np.linalg.eigvalsh(I).min() >= -1e-12 * np.trace(I)
        assert abs(I[0, 1] - r["trace"]["a"] / (2 * theta[0])) < 1e-15 * abs(I[0, 1]) + 1e-300


def test_invariances(oracle_mod):
    locs, z = _data(50, 9)
    theta = np.array([1.3, 0.07, 1.1])
    base = oracle_mod.evaluate(locs, z, theta)
    perm = np.random.default_rng(4).permutation(50)
    p = oracle_mod.evaluate(locs[perm], z[perm], theta)
    assert abs(p["loglik"] - base["loglik"]) < 1e-11 * abs(base["loglik"])
    np.testing.assert_allclose(p["score"], base["score"], rtol=1e-9, atol=1e-9)
    # (s, alpha) -> (c s, c alpha): l, l_sigma2, l_nu unchanged, l_alpha / c
    c = 3.0
    s = oracle_mod.evaluate(locs * c, z, theta * np.array([1, c, 1]))
    assert abs(s["loglik"] - base["loglik"]) < 1e-11 * abs(base["loglik"])
    np.testing.assert_allclose(s["score"], base["score"] / np.array([1, c, 1]), rtol=1e-9,
                               atol=1e-9)
    # (Z, sigma2) -> (c Z, c^2 sigma2): l shifts by -n log c
    v = oracle_mod.evaluate(locs, z * c, theta * np.array([c * c, 1, 1]))
    assert abs(v["loglik"] - (base["loglik"] - 50 * math.log(c))) < 1e-11 * abs(base["loglik"])


@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.5), (0.7, 0.04, 1.7), (1.5, 0.15, 0.3)])
def test_score_by_central_differences(oracle_mod, theta):
    locs, z = _data(150, 21)
    theta = np.array(theta)
    r = oracle_mod.evaluate(locs, z, theta)
    for i in range(3):
        d = 1e-6 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += d
        tm[i] -= d
        fd = (oracle_mod.loglik(locs, z, tp)["loglik"] - oracle_mod.loglik(locs, z, tm)["loglik"]) / (2 * d)
        # term scale of Eq. (2): the score is a difference of two such terms
        if i == 0:
            scale = (r["quad"] + 150) / (2 * theta[0])
        else:
            k = "a" if i == 1 else "n"
            scale = 0.5 * (abs(r["trace"][k]) + abs(r["wSw"][k]))
        assert abs(fd - r["score"][i]) <= 1e-7 * scale, (i, fd, r["score"][i], scale)


def test_loglik_matches_eval(oracle_mod):
    locs, z = _data(90, 2)
    a = oracle_mod.loglik(locs, z, (1.0, 0.1, 0.5))
    b = oracle_mod.evaluate(locs, z, (1.0, 0.1, 0.5))
    assert a["loglik"] == b["loglik"] and a["logdet"] == b["logdet"]


def test_not_positive_definite(oracle_mod):
    locs = np.array([[0.1, 0.1], [0.1, 0.1], [0.5, 0.2]])   # duplicated location
    with pytest.raises(oracle_mod.NotPositiveDefinite):
        oracle_mod.loglik(locs, np.ones(3), (1.0, 0.1, 0.5))
    with pytest.raises(ValueError):
        oracle_mod.loglik(locs[1:], np.ones(2), (1.0, -0.1, 0.5))


def test_monte_carlo_score_moments(oracle_mod):
    """E[score] = 0 and Cov[score] = I(theta) under the model (Eq. (3))."""
    n, reps = 12, 3000
    gen = np.random.default_rng(123)
    locs = gen.random((n, 2))
    theta = (1.0, 0.3, 0.8)
    (S,) = oracle_mod.cov_matrices(locs, theta, which=("S",))
    L = np.linalg.cholesky(S)
    scores = np.array([oracle_mod.evaluate(locs, L @ gen.standard_normal(n), theta)["score"]
                       for _ in range(reps)])
    I = oracle_mod.evaluate(locs, np.zeros(n), theta)["fisher"]
    se = np.sqrt(np.diag(I) / reps)
    assert np.all(np.abs(scores.mean(axis=0)) < 4.5 * se)
    cov = np.cov(scores.T)
    d = np.sqrt(np.diag(I))
    corr_err = np.abs(cov - I) / np.outer(d, d)
    assert corr_err.max() < 0.12
