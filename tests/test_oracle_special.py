"""Pins of the oracle's special functions and Matern entries against
mathematics that does not depend on the oracle: closed forms, DLMF identities,
SciPy's AMOS Bessel routines and mpmath at 30+ digits.

Matern covariance: Section 2.1.  C_alpha: Section 2.2.  C_nu: the exact
nu-derivative that Supplement A approximates.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.special as sp

XS = [1e-8, 1e-5, 1e-3, 0.02, 0.3, 1.0, 2.7, 8.0, 15.0, 29.0, 44.0, 61.0, 120.0, 400.0]


def rel(a, b):
    return abs(a - b) / abs(b)


# --------------------------------------------------------------- K_mu values
@pytest.mark.parametrize("x", XS)
def test_k_half_integer_closed_forms(oracle_mod, x):
    """K_{1/2}, K_{3/2}, K_{5/2} (DLMF 10.39.2 and the order recurrence)."""
    base = math.sqrt(math.pi / (2 * x))
    forms = {0.5: 1.0, 1.5: 1.0 + 1.0 / x, 2.5: 1.0 + 3.0 / x + 3.0 / x ** 2}
    for mu, poly in forms.items():
        got = oracle_mod.bessel_k_scaled(mu, x)
        assert rel(got, base * poly) < 1e-14, (mu, x)
        assert rel(oracle_mod.bessel_k_scaled(-mu, x), base * poly) < 1e-14   # K_{-mu} = K_mu


def test_k_against_scipy_amos(oracle_mod):
    gen = np.random.default_rng(7)
    worst = 0.0
    for _ in range(400):
        mu = gen.uniform(-2.0, 4.0)
        x = 10 ** gen.uniform(-6, 2.6)
        worst = max(worst, rel(oracle_mod.bessel_k_scaled(mu, x), sp.kve(mu, x)))
    assert worst < 5e-14


def test_k_against_mpmath(oracle_mod):
    mp.mp.dps = 35
    for mu in (0.05, 0.37, 0.8, 1.0, 1.93, 3.3, -0.6):
        for x in (1e-7, 4e-3, 0.9, 6.5, 33.0, 250.0):
            ref = float(mp.besselk(mu, x) * mp.e ** x)
            assert rel(oracle_mod.bessel_k_scaled(mu, x), ref) < 2e-15, (mu, x)


@pytest.mark.parametrize("nu", [0.13, 0.5, 0.77, 1.25, 2.6])
def test_k_order_recurrence(oracle_mod, nu):
    """K_{nu+1}(x) = K_{nu-1}(x) + (2 nu / x) K_nu(x)  (DLMF 10.29.1)."""
    for x in (1e-3, 0.4, 3.0, 20.0, 90.0):
        k = lambda m: oracle_mod.bessel_k_scaled(m, x)
        lhs = k(nu + 1)
        rhs = k(nu - 1) + 2 * nu / x * k(nu)
        assert rel(lhs, rhs) < 1e-14


# ----------------------------------------------------------- dK_mu / dmu
@pytest.mark.parametrize("x", XS[:-1])
def test_dk_closed_forms(oracle_mod, x):
    """d/dnu K_nu at nu = 1/2 (DLMF 10.38.7), nu = 1 (K_0(x)/x), nu = 3/2 (the
    differentiated order recurrence), and nu = 0 (K is even in its order)."""
    e1 = sp.exp1(2 * x) * math.exp(2 * x)          # e^{2x} E_1(2x), scaled
    base = math.sqrt(math.pi / (2 * x))
    half = base * e1
    three_half = base * ((1.0 / x - 1.0) * e1 + 2.0 / x)
    one = sp.k0e(x) / x
    assert rel(oracle_mod.bessel_dk_dnu_scaled(0.5, x), half) < 1e-13
    assert rel(oracle_mod.bessel_dk_dnu_scaled(1.0, x), one) < 1e-13
    assert rel(oracle_mod.bessel_dk_dnu_scaled(1.5, x), three_half) < 1e-13
    assert oracle_mod.bessel_dk_dnu_scaled(0.0, x) == 0.0


def test_dk_against_mpmath(oracle_mod):
    mp.mp.dps = 40
    for nu in (0.05, 0.3, 0.9, 1.0, 2.2, 3.0):
        for x in (1e-6, 2e-2, 0.7, 5.0, 27.0, 140.0):
            ref = float(mp.diff(lambda m: mp.besselk(m, x), nu) * mp.e ** x)
            assert rel(oracle_mod.bessel_dk_dnu_scaled(nu, x), ref) < 5e-15, (nu, x)


def test_digamma(oracle_mod):
    euler = 0.5772156649015329
    assert abs(oracle_mod.digamma(1.0) + euler) < 1e-15
    assert abs(oracle_mod.digamma(0.5) + euler + 2 * math.log(2)) < 1e-15
    for v in np.linspace(0.01, 30, 200):
        assert abs(oracle_mod.digamma(v) - sp.digamma(v)) <= 1e-14 * max(1.0, abs(sp.digamma(v)))


# --------------------------------------------------------------- Matern C
THETA_SHAPES = [(1.0, 0.1), (2.3, 0.037), (0.4, 1.7)]


@pytest.mark.parametrize("s2,a", THETA_SHAPES)
def test_matern_half_integer_closed_forms(oracle_mod, s2, a):
    """C and dC/dalpha at nu = 1/2, 3/2, 5/2 in closed form."""
    h = np.array([1e-9, 1e-4, 0.003, 0.05, 0.2, 0.9, 1.41]) * max(a, 0.1) * 10
    x = h / a
    e = np.exp(-x)
    forms = {
        0.5: (e, x * e),
        1.5: ((1 + x) * e, x ** 2 * e),
        2.5: ((1 + x + x ** 2 / 3) * e, (x ** 2 + x ** 3) * e / 3),
    }
    for nu, (c, ca) in forms.items():
        got_c, got_ca, _ = oracle_mod.matern_entries(h, (s2, a, nu))
        np.testing.assert_allclose(got_c, s2 * c, rtol=2e-14, atol=0)
        np.testing.assert_allclose(got_ca, s2 / a * ca, rtol=2e-14, atol=1e-300)


@pytest.mark.parametrize("s2,a", THETA_SHAPES)
def test_matern_dnu_half_closed_form(oracle_mod, s2, a):
    """C_nu at nu = 1/2: sigma2 [e^{-x}(gamma + log 2x) + e^{x} E_1(2x)]."""
    h = np.array([1e-6, 1e-3, 0.02, 0.3, 1.0, 1.4]) * a * 5
    x = h / a
    euler = 0.5772156649015329
    ref = s2 * np.exp(-x) * ((euler + np.log(2 * x)) + sp.exp1(2 * x) * np.exp(2 * x))
    _, _, cn = oracle_mod.matern_entries(h, (s2, a, 0.5))
    np.testing.assert_allclose(cn, ref, rtol=1e-13, atol=1e-14 * s2)


def test_matern_at_zero_distance(oracle_mod):
    for theta in ((1.0, 0.1, 0.5), (3.0, 0.02, 2.7), (0.2, 4.0, 0.05)):
        c, ca, cn = oracle_mod.matern_entries([0.0], theta)
        assert c[0] == theta[0] and ca[0] == 0.0 and cn[0] == 0.0
    # small-x expansion: C / sigma2 = 1 - Gamma(1-nu)/Gamma(1+nu) (x/2)^(2 nu) + O(x^2)
    # for 0 < nu < 1 (from K_nu = pi (I_{-nu} - I_nu) / (2 sin(nu pi))), and
    # C / sigma2 = 1 - x^2 / (4 (nu - 1)) + o(x^2) for nu > 1.
    for nu in (0.05, 0.3, 0.72):
        for x in (1e-12, 1e-9, 1e-6):
            c, _, _ = oracle_mod.matern_entries([x * 0.1], (1.0, 0.1, nu))
            ref = 1 - sp.gamma(1 - nu) / sp.gamma(1 + nu) * (x / 2) ** (2 * nu)
            assert abs(c[0] - ref) < 1e-11 + x ** 2, (nu, x)
    for nu in (1.6, 2.7):
        x = 1e-4
        c, _, _ = oracle_mod.matern_entries([x * 0.1], (1.0, 0.1, nu))
        assert abs((1 - c[0]) / (x * x / (4 * (nu - 1))) - 1) < 1e-3


def _scipy_matern(h, s2, a, nu):
    x = h / a
    return s2 * 2 ** (1 - nu) / sp.gamma(nu) * x ** nu * sp.kv(nu, x)


@pytest.mark.parametrize("nu", [0.08, 0.37, 0.5, 1.0, 1.3, 2.2, 3.0])
def test_matern_derivatives_by_finite_differences(oracle_mod, nu):
    """C_alpha and C_nu against central differences of SciPy's Matern."""
    s2, a = 1.3, 0.11
    h = np.array([1e-4, 0.01, 0.05, 0.11, 0.3, 0.8])
    _, ca, cn = oracle_mod.matern_entries(h, (s2, a, nu))
    da, dn = 1e-5 * a, 1e-5 * nu
    fa = (_scipy_matern(h, s2, a + da, nu) - _scipy_matern(h, s2, a - da, nu)) / (2 * da)
    fn = (_scipy_matern(h, s2, a, nu + dn) - _scipy_matern(h, s2, a, nu - dn)) / (2 * dn)
    np.testing.assert_allclose(ca, fa, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(cn, fn, rtol=1e-6, atol=1e-9)


def test_matern_dnu_against_mpmath(oracle_mod):
    mp.mp.dps = 40
    s2, a = 0.7, 0.05

    def C(h, nu):
        x = mp.mpf(h) / a
        return s2 * 2 ** (1 - nu) / mp.gamma(nu) * x ** nu * mp.besselk(nu, x)

    for nu in (0.11, 0.5, 0.93, 1.0, 2.5):
        for h in (1e-5, 2e-3, 0.04, 0.2, 0.9):
            ref = float(mp.diff(lambda v: C(h, v), nu))
            ca_ref = float(mp.diff(lambda al: s2 * 2 ** (1 - nu) / mp.gamma(nu)
                                   * (h / al) ** nu * mp.besselk(nu, h / al), a))
            _, ca, cn = oracle_mod.matern_entries([h], (s2, a, nu))
            assert abs(cn[0] - ref) <= max(1e-13 * abs(ref), 1e-14 * s2), (nu, h)
            assert abs(ca[0] - ca_ref) <= max(1e-13 * abs(ca_ref), 1e-300), (nu, h)


def test_matern_range_scaling_identity(oracle_mod):
    """alpha dC/dalpha = -h dC/dh (C depends on h/alpha only)."""
    s2, a = 1.0, 0.2
    for nu in (0.3, 1.1, 2.4):
        h = np.array([0.01, 0.1, 0.4, 1.0])
        _, ca, _ = oracle_mod.matern_entries(h, (s2, a, nu))
        dh = 1e-6 * h
        cp, _, _ = oracle_mod.matern_entries(h + dh, (s2, a, nu))
        cm, _, _ = oracle_mod.matern_entries(h - dh, (s2, a, nu))
        np.testing.assert_allclose(a * ca, -h * (cp - cm) / (2 * dh), rtol=2e-6)
