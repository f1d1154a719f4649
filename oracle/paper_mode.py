"""Paper mode for the oracle: Sigma_nu by the paper's own numerical scheme for
d/dnu [x^nu K_nu(x)] (Supplementary Material A), instead of the exact
derivative the rest of the oracle uses.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The scheme picks one of five cases per entry (x = h / alpha):
  1. x = 0: the derivative is 0;
  2. x < 8.5 and nu at least 1e-6 from the nearest integer: the power series
     of K_nu (two Gamma-weighted series in (x/2)^2) differentiated term by term,
     truncated after 20 terms;
  3. 8.5 <= x < 30: the uniform (Debye) expansion of K_nu(nu z), z = x / nu,
     differentiated in nu, truncated after 12 terms for x < 15 and 8 terms
     beyond;
  4. x >= 30 and nu + 1/2 at least 1e-6 from the nearest integer: the Hankel
     expansion of K_nu, differentiated in nu, truncated after 5 terms;
  5. otherwise: a central difference in nu with lag 1e-9 of x^nu K_nu(x), the
     latter from the accurate quadrature of the oracle.
Readings (listed in the design notes): "up to the K-th term" is K terms,
k = 0..K-1; the difference in case 5 is central; Sigma_nu itself adds the
derivative of the prefactor 2^(1-nu) / Gamma(nu), which is exact:
  C_nu = sigma2 c_nu [ d/dnu(x^nu K_nu) - (log 2 + psi(nu)) x^nu K_nu ].
The Debye polynomials U_k are built from their defining recursion
  U_0 = 1,  U_{k+1}(p) = p^2 (1 - p^2) U_k'(p) / 2 + (1/8) int_0^p (1 - 5 t^2) U_k(t) dt
with exact polynomial arithmetic (numpy.polynomial), not from the
coefficient recurrence printed with it.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import polynomial as P
from scipy.special import digamma as _psi

_U_CACHE: list = []


def debye_u(k: int) -> np.ndarray:
    """Coefficients (ascending powers of p) of the Debye polynomial U_k."""
    while len(_U_CACHE) <= k:
        if not _U_CACHE:
            _U_CACHE.append(np.array([1.0]))
            continue
        u = _U_CACHE[-1]
        term1 = 0.5 * P.polymul([0.0, 0.0, 1.0, 0.0, -1.0], P.polyder(u))   # p^2 (1 - p^2) U'/2
        term2 = 0.125 * P.polyint(P.polymul([1.0, 0.0, -5.0], u))          # lower limit 0
        _U_CACHE.append(P.polyadd(term1, term2))
    return _U_CACHE[k]


def _xnuk(x: float, nu: float, bessel_k) -> float:
    return x ** nu * bessel_k(nu, x)


def _case2(x: float, nu: float, terms: int = 20) -> float:
    """Term-by-term derivative of the power series of x^nu K_nu(x)."""
    g_nu, g_mnu = math.gamma(nu), math.gamma(-nu)
    psi_nu, psi_mnu = _psi(nu), _psi(-nu)
    tot = 0.0
    gk_m, gk_p = 1.0, 1.0        # g_k(-nu), g_k(nu)
    dk_m, dk_p = 0.0, 0.0        # d_k(-nu), d_k(nu)
    fact = 1.0
    for k in range(terms):
        if k >= 1:
            gk_m /= (-nu + k)
            gk_p /= (nu + k)
            dk_m -= 1.0 / (-nu + k)
            dk_p -= 1.0 / (nu + k)
            fact *= k
        pre = (x / 2.0) ** (2 * k) / (2.0 * fact)
        a = 2.0 ** nu * (math.log(2.0) + psi_nu - dk_m) * g_nu * gk_m
        b = (2.0 ** -nu * x ** (2 * nu) * (-math.log(2.0) + 2.0 * math.log(x) - psi_mnu + dk_p)
             * g_mnu * gk_p)
        tot += pre * (a + b)
    return tot


def _case3(x: float, nu: float) -> float:
    """Nu-derivative of the uniform expansion of K_nu(nu z) at z = x / nu."""
    terms = 12 if x < 15.0 else 8
    z = x / nu
    q = 1.0 + z * z
    sq = math.sqrt(q)
    p = 1.0 / sq
    eta = sq + math.log(z / (1.0 + sq))
    g = x ** nu * math.sqrt(math.pi / (2.0 * nu)) * math.exp(-nu * eta) / q ** 0.25
    s0 = s1 = s2 = 0.0
    for k in range(terms):
        u = debye_u(k)
        uk = P.polyval(p, u)
        duk = P.polyval(p, P.polyder(u)) if k > 0 else 0.0
        sgn = -1.0 if k % 2 else 1.0
        s0 += sgn * nu ** -k * uk
        s1 += sgn * k * nu ** (-k - 1) * uk
        s2 += sgn * nu ** -k * duk
    lead = math.log(nu) + math.log(1.0 + sq) - 1.0 / (2.0 * nu * q)
    return lead * g * s0 - g * s1 + (x * x / nu ** 3) * q ** -1.5 * g * s2


def _case4(x: float, nu: float, terms: int = 5) -> float:
    """Nu-derivative of the Hankel expansion of x^nu K_nu(x)."""
    tot = 0.0
    a, b = 1.0, 0.0
    for k in range(terms):
        if k >= 1:
            f = 4.0 * nu * nu - (2 * k - 1) ** 2
            a *= f / (8.0 * k)
            b += 8.0 * nu / f
        tot += x ** -k * (math.log(x) + b) * a
    return math.sqrt(math.pi / 2.0) * x ** (nu - 0.5) * math.exp(-x) * tot


def case_of(x: float, nu: float) -> int:
    if x == 0.0:
        return 1
    if x < 8.5 and abs(nu - round(nu)) > 1e-6:
        return 2
    if 8.5 <= x < 30.0:
        return 3
    if x >= 30.0 and abs((nu + 0.5) - round(nu + 0.5)) > 1e-6:
        return 4
    return 5


def dxnuk_dnu(x: float, nu: float, bessel_k) -> float:
    """d/dnu [x^nu K_nu(x)] by the case scheme; bessel_k(mu, x) is the
    accurate value routine used by case 5."""
    c = case_of(x, nu)
    if c == 1:
        return 0.0
    if c == 2:
        return _case2(x, nu)
    if c == 3:
        return _case3(x, nu)
    if c == 4:
        return _case4(x, nu)
    lag = 1e-9
    return (_xnuk(x, nu + lag, bessel_k) - _xnuk(x, nu - lag, bessel_k)) / (2.0 * lag)


def sigma_nu_entries(h, theta, bessel_k) -> np.ndarray:
    """Paper-mode dC/dnu at distances h."""
    s2, a, nu = (float(t) for t in theta)
    cnu = 2.0 ** (1.0 - nu) / math.gamma(nu)
    lp = math.log(2.0) + _psi(nu)
    out = np.empty(np.size(h))
    for i, hh in enumerate(np.ravel(h)):
        x = float(hh) / a
        if x == 0.0:
            out[i] = 0.0
            continue
        d = dxnuk_dnu(x, nu, bessel_k)
        out[i] = s2 * cnu * (d - lp * _xnuk(x, nu, bessel_k))
    return out
