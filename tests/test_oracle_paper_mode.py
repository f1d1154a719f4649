"""Pins of the oracle's paper mode (the case scheme of Supplementary A for
d/dnu [x^nu K_nu(x)]):

  * the Debye polynomials built from their defining recursion equal the
    published U_1, U_2, U_3 (DLMF 10.41.10);
  * the case selection follows the order of the scheme's tests;
  * each case agrees with the exact derivative x^nu (log x K_nu + dK_nu/dnu)
    of the oracle within the truncation / differencing error of that case:
    case 2 (20 terms) <= 5e-6 for x < 8.5 and <= 1e-10 for x <= 3, case 3
    (12 / 8 terms) <= 5e-8, case 4 (5 terms, x >= 30) <= 1e-7, case 5 (central
    difference, lag 1e-9) <= 2e-6;
  * Sigma_nu in paper mode is the exact prefactor term plus the scheme's
    derivative, and vanishes on the diagonal;
  * the dense paper-mode Sigma_nu of three points at hand-computed distances
    holds the scheme's entry of each pair, symmetric with a zero diagonal;
  * Eqs. (1)-(3) with a pair-by-pair paper-mode Sigma_nu and a 30-digit
    inverse and determinant (n = 20) equal the oracle's paper-mode evaluation
    and adjoint score.
"""
import math

import numpy as np
import pytest

from oracle import paper_mode as pm


def test_debye_polynomials():
    np.testing.assert_allclose(pm.debye_u(1), np.array([0, 3, 0, -5]) / 24, rtol=1e-15)
    np.testing.assert_allclose(pm.debye_u(2), np.array([0, 0, 81, 0, -462, 0, 385]) / 1152,
                               rtol=1e-15)
    u3 = np.array([0, 0, 0, 30375, 0, -369603, 0, 765765, 0, -425425]) / 414720
    np.testing.assert_allclose(pm.debye_u(3), u3, rtol=1e-14)


def test_case_selection():
    assert pm.case_of(0.0, 0.7) == 1
    assert pm.case_of(1.0, 0.7) == 2
    assert pm.case_of(1.0, 1.0 + 5e-7) == 5        # nu within 1e-6 of an integer, x < 8.5
    assert pm.case_of(1.0, 1.0 + 2e-6) == 2
    assert pm.case_of(8.5, 1.0) == 3
    assert pm.case_of(29.99, 0.5) == 3
    assert pm.case_of(30.0, 0.7) == 4
    assert pm.case_of(30.0, 0.5) == 5              # nu + 1/2 an integer, x >= 30
    assert pm.case_of(40.0, 1.5 + 5e-7) == 5


def _exact(oracle_mod, x, nu):
    return x ** nu * (math.log(x) * oracle_mod.bessel_k(nu, x) + oracle_mod.bessel_dk_dnu(nu, x))


@pytest.mark.parametrize("nu", [0.3, 0.5, 0.9, 1.0, 1.3, 1.5, 2.7])
def test_cases_against_exact(oracle_mod, nu):
    for x in [0.05, 0.5, 1.0, 3.0, 5.0, 8.4, 8.6, 12.0, 16.0, 29.0, 31.0, 45.0]:
        c = pm.case_of(x, nu)
        got = pm.dxnuk_dnu(x, nu, oracle_mod.bessel_k)
        want = _exact(oracle_mod, x, nu)
        rel = abs(got - want) / abs(want)
        bound = {2: 1e-10 if x <= 3.0 else 5e-6, 3: 5e-8, 4: 1e-7, 5: 2e-6}[c]
        assert rel <= bound, (nu, x, c, rel)


def test_sigma_nu_paper_mode(oracle_mod):
    theta = (1.3, 0.1, 0.8)
    h = np.array([0.0, 0.003, 0.05, 0.3, 0.9, 2.0, 4.0])
    got = pm.sigma_nu_entries(h, theta, oracle_mod.bessel_k)
    _, _, exact = oracle_mod.matern_entries(h, theta)
    assert got[0] == 0.0
    # same prefactor handling: the difference is c_nu sigma2 times the scheme's error
    for i in range(1, h.size):
        x = h[i] / theta[1]
        err = abs(pm.dxnuk_dnu(x, theta[2], oracle_mod.bessel_k) - _exact(oracle_mod, x, theta[2]))
        cnu = 2 ** (1 - theta[2]) / math.gamma(theta[2])
        assert abs(got[i] - exact[i]) <= theta[0] * cnu * err * (1 + 1e-6) + 1e-15 * theta[0]


@pytest.mark.parametrize("theta", [(1.3, 0.05, 0.8), (0.7, 0.05, 1.0)])
def test_paper_sigma_nu_matrix_n3(oracle_mod, theta):
    """The dense paper-mode Sigma_nu of three points at hand-computed distances
    (a 3-4-5 triangle: 0.3, 0.4, 0.5, i.e. x = 6, 8, 10 at alpha = 0.05, cases
    2 and 3, or case 5 at integer nu): each off-diagonal entry is the scheme's
    value at that pair's distance, the matrix is symmetric, the diagonal zero."""
    locs = np.array([[0.0, 0.0], [0.3, 0.0], [0.0, 0.4]])
    S = oracle_mod._paper_sigma_nu(locs, theta)
    assert S.shape == (3, 3)
    np.testing.assert_array_equal(np.diag(S), 0.0)
    np.testing.assert_array_equal(S, S.T)
    for (a, b), h in (((1, 0), 0.3), ((2, 0), 0.4), ((2, 1), 0.5)):
        want = pm.sigma_nu_entries(np.array([h]), theta, oracle_mod.bessel_k)[0]
        assert want != 0.0
        assert abs(S[a, b] - want) <= 1e-13 * abs(want), (a, b, S[a, b], want)


def _brute_force_given(S, derivs, z, dps=30):
    """Eqs. (1)-(3) literally from given matrices, with a 30-digit inverse and
    determinant; derivs = (Sigma_sigma2, Sigma_alpha, Sigma_nu)."""
    import mpmath as mp

    mp.mp.dps = dps
    n = z.size
    M = mp.matrix(S.tolist())
    Minv = M ** -1
    Zm = mp.matrix(z.tolist())
    ll = -mp.mpf(n) / 2 * mp.log(2 * mp.pi) - mp.log(mp.det(M)) / 2 - (Zm.T * Minv * Zm)[0] / 2
    Dm = [mp.matrix(D.tolist()) for D in derivs]
    A = [Minv * D for D in Dm]
    w = Minv * Zm
    score = [-sum(Ai[k, k] for k in range(n)) / 2 + (w.T * D * w)[0] / 2 for Ai, D in zip(A, Dm)]
    fisher = np.array([[float(sum((A[i] * A[j])[k, k] for k in range(n)) / 2) for j in range(3)]
                       for i in range(3)])
    return float(ll), np.array([float(s) for s in score]), fisher


@pytest.mark.parametrize("theta", [(1.1, 0.1, 0.8), (0.9, 0.08, 1.0)])
def test_paper_mode_evaluation_brute_force_n20(oracle_mod, theta):
    """Eqs. (1)-(3) with the paper-mode Sigma_nu assembled pair by pair here
    (math.hypot distances, one scheme call per pair) against the oracle's
    evaluation and adjoint score in paper mode."""
    import synth

    locs, z, _ = synth.dataset(20, (1.0, 0.1, 0.5), 17)
    n = z.size
    S, Sa = oracle_mod.cov_matrices(locs, theta, which=("S", "Sa"))
    Sn = np.zeros((n, n))
    for a in range(n):
        for b in range(a):
            h = math.hypot(locs[a, 0] - locs[b, 0], locs[a, 1] - locs[b, 1])
            Sn[a, b] = Sn[b, a] = pm.sigma_nu_entries(np.array([h]), theta, oracle_mod.bessel_k)[0]
    ll, score, fisher = _brute_force_given(S, (S / theta[0], Sa, Sn), z)
    r = oracle_mod.evaluate(locs, z, theta, sigma_nu="paper")
    assert abs(r["loglik"] - ll) <= 1e-12 * abs(ll)
    scale = np.abs(score) + np.abs(np.diag(fisher)) + 1.0
    np.testing.assert_allclose(r["score"], score, rtol=0, atol=1e-11 * scale.max())
    np.testing.assert_allclose(r["fisher"], fisher, rtol=1e-11)
    adj = oracle_mod.adjoint_score(locs, z, theta, sigma_nu="paper")
    np.testing.assert_allclose(adj["score"], score, rtol=0, atol=1e-11 * scale.max())
    # the exact-mode evaluation differs only through Sigma_nu
    e = oracle_mod.evaluate(locs, z, theta)
    assert e["loglik"] == r["loglik"] and e["score"][0] == r["score"][0]
