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
    derivative, and vanishes on the diagonal.
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
