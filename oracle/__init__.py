"""Plain FP64 CPU oracle for the exact Matern log-likelihood, score and Fisher
information (Hong, Abdulah, Genton & Sun, Sections 2.1-2.2, Algorithms 2-3)
and for the Fisher-BT fit (Algorithm 1, Table 1, Eq. (4)).

TEST INFRASTRUCTURE ONLY.  The oracle is what the HIP library is checked
against.  It shares no code with the product: no kernels, headers, helpers,
tables or constant generators, and neither imports the other.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it.

Layout:
  matern_oracle.c  per-entry Matern C, dC/dalpha, dC/dnu via trapezoid quadrature
                   of the integral form of K_nu (compiled by ``build()``)
  __init__.py      Eqs. (1)-(3) from one Cholesky and one joint solve (LAPACK),
                   and the adjoint form of Eq. (2) with an explicit inverse
  fisher_bt.py     Algorithm 1 (L9 start, Fisher scoring, relaxed Armijo
                   backtracking, Nelder-Mead fallback)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.linalg

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "matern_oracle.c")
_SO = os.path.join(_HERE, "libmatern_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (IEEE FP64, no fast-math)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        d, i64, p = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
        lib.oracle_digamma.restype = d
        lib.oracle_digamma.argtypes = [d]
        for f in (lib.oracle_bessel_k_scaled, lib.oracle_bessel_dk_scaled):
            f.restype = d
            f.argtypes = [d, d]
        lib.oracle_matern_entries.restype = None
        lib.oracle_matern_entries.argtypes = [i64, p, d, d, d, p, p, p]
        lib.oracle_cov_matrices.restype = None
        lib.oracle_cov_matrices.argtypes = [i64, p, d, d, d, p, p, p]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class NotPositiveDefinite(ArithmeticError):
    """Sigma(theta) failed the Cholesky factorisation."""


# --------------------------------------------------------------------------
# Special functions (DLMF 10.32.9 and its order derivative)
# --------------------------------------------------------------------------
def digamma(v: float) -> float:
    return _load().oracle_digamma(float(v))


def bessel_k(mu: float, x: float) -> float:
    """K_mu(x) for x > 0."""
    return _load().oracle_bessel_k_scaled(float(mu), float(x)) * np.exp(-x)


def bessel_k_scaled(mu: float, x: float) -> float:
    """e^x K_mu(x) for x > 0."""
    return _load().oracle_bessel_k_scaled(float(mu), float(x))


def bessel_dk_dnu(mu: float, x: float) -> float:
    """d K_mu(x) / d mu for x > 0."""
    return _load().oracle_bessel_dk_scaled(float(mu), float(x)) * np.exp(-x)


def bessel_dk_dnu_scaled(mu: float, x: float) -> float:
    return _load().oracle_bessel_dk_scaled(float(mu), float(x))


# --------------------------------------------------------------------------
# Matern covariance and its derivatives (Section 2.1, Section 2.2)
# --------------------------------------------------------------------------
def matern_entries(h, theta):
    """(C, C_alpha, C_nu) at distances h (array) for theta = (sigma2, alpha, nu)."""
    h = np.ascontiguousarray(np.asarray(h, dtype=np.float64).ravel())
    s2, a, nu = (float(t) for t in theta)
    c, ca, cn = (np.empty_like(h) for _ in range(3))
    _load().oracle_matern_entries(h.size, _ptr(h), s2, a, nu, _ptr(c), _ptr(ca), _ptr(cn))
    return c, ca, cn


def cov_matrices(locs, theta, which=("S", "Sa", "Sn")):
    """Dense Sigma, Sigma_alpha, Sigma_nu (n x n) for locations (n x 2)."""
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    n = locs.shape[0]
    out = {k: (np.empty((n, n)) if k in which else None) for k in ("S", "Sa", "Sn")}
    s2, a, nu = (float(t) for t in theta)
    _load().oracle_cov_matrices(n, _ptr(locs), s2, a, nu,
                                _ptr(out["S"]), _ptr(out["Sa"]), _ptr(out["Sn"]))
    return tuple(out[k] for k in which)


# --------------------------------------------------------------------------
# The Gaussian likelihood and its first two moments in theta (Eqs. (1)-(3))
# --------------------------------------------------------------------------
def _check_theta(theta):
    theta = np.asarray(theta, dtype=np.float64)
    if theta.shape != (3,) or not np.all(np.isfinite(theta)) or np.any(theta <= 0):
        raise ValueError("theta must be three finite positive numbers (sigma2, alpha, nu)")
    return theta


def _spd_solve(S, rhs):
    """log det S and S^{-1} rhs for a symmetric positive definite S.

    Both come from one LAPACK Cholesky factorisation S = C C^T (dpotrf; the
    determinant is the squared product of C's diagonal) and dpotrs for every
    column of ``rhs`` at once.  A failed factorisation raises
    NotPositiveDefinite."""
    try:
        c = scipy.linalg.cho_factor(S, lower=True, check_finite=False)
    except np.linalg.LinAlgError as e:
        raise NotPositiveDefinite(str(e)) from None
    logdet = 2.0 * float(np.sum(np.log(np.diag(c[0]))))
    return logdet, scipy.linalg.cho_solve(c, rhs, check_finite=False)


def _gaussian_loglik(n, logdet, quad):
    """Eq. (1): the zero-mean Gaussian log-density of Z, from log|Sigma| and
    the quadratic form Z^T Sigma^{-1} Z."""
    return -0.5 * n * np.log(2 * np.pi) - 0.5 * logdet - 0.5 * quad


def trace_product_frobenius(A, B):
    """trace(AB) via the Frobenius identity of Eq. (5)."""
    return 0.5 * (np.sum((A + B.T) ** 2) - np.sum(A ** 2) - np.sum(B ** 2))


def loglik(locs, z, theta):
    """Eq. (1) at theta.  Returns dict(loglik, logdet, quad) with
    quad = Z^T Sigma^{-1} Z."""
    theta = _check_theta(theta)
    z = np.asarray(z, dtype=np.float64)
    (S,) = cov_matrices(locs, theta, which=("S",))
    logdet, w = _spd_solve(S, z)
    quad = float(z @ w)
    return {"loglik": float(_gaussian_loglik(z.size, logdet, quad)), "logdet": logdet,
            "quad": quad}


def _paper_sigma_nu(locs, theta):
    """Dense Sigma_nu whose entries follow the paper's case scheme for the
    order derivative (Supplementary A, ``oracle.paper_mode``): the entry of
    each pair j > k at its Euclidean distance, mirrored to k > j; the diagonal
    (zero distance) is zero."""
    from . import paper_mode

    locs = np.asarray(locs, dtype=np.float64)
    n = locs.shape[0]
    i, j = np.tril_indices(n, -1)
    h = np.hypot(locs[i, 0] - locs[j, 0], locs[i, 1] - locs[j, 1])
    v = paper_mode.sigma_nu_entries(h, theta, bessel_k)
    Sn = np.zeros((n, n))
    Sn[i, j] = v
    Sn[j, i] = v
    return Sn


def evaluate(locs, z, theta, sigma_nu="exact", progress=None):
    """Log-likelihood (Eq. (1)), score (Eq. (2)) and expected Fisher
    information (Eq. (3)) over theta = (sigma2, alpha, nu).

    One Cholesky of Sigma solves Sigma X = [Z | Sigma_alpha | Sigma_nu]; the
    first column is w = Sigma^{-1} Z, the other blocks are
    A_i = Sigma^{-1} Sigma_i.  Then, for i in {alpha, nu},

        dl/dtheta_i = -tr(A_i) / 2 + w^T Sigma_i w / 2,   I_ij = tr(A_i A_j) / 2.

    The covariance is proportional to sigma2, so Sigma_{sigma2} = Sigma / sigma2
    and A_{sigma2} = I / sigma2, which gives dl/dsigma2 = (Z^T w - n) / (2 sigma2),
    I_{sigma2,sigma2} = n / (2 sigma2^2) and I_{sigma2,i} = tr(A_i) / (2 sigma2).

    Besides the results it returns the intermediate traces and quadratic
    forms, and every alpha/nu Fisher entry twice: tr(A_i A_j) by the
    Frobenius identity of Eq. (5) and by the direct sum sum_jk (A_i)_jk (A_j)_kj
    (the entry reported is the former).  ``sigma_nu="paper"`` replaces the
    exact Sigma_nu with the paper's approximation of it (Supplementary A).
    ``progress``, if given, is called with a short text after the matrices
    are generated and after the joint solve (long evaluations report there).
    """
    theta = _check_theta(theta)
    s2 = theta[0]
    z = np.asarray(z, dtype=np.float64)
    n = z.size
    S, Sa, Sn = cov_matrices(locs, theta)
    if sigma_nu == "paper":
        Sn = _paper_sigma_nu(locs, theta)
    deriv = {"a": Sa, "n": Sn}
    if progress:
        progress("covariance and derivative matrices generated")
    logdet, X = _spd_solve(S, np.hstack([z[:, None], Sa, Sn]))
    del S
    if progress:
        progress("Cholesky factorisation and joint solve done")
    w = X[:, 0]
    A = {"a": X[:, 1:n + 1], "n": X[:, n + 1:]}
    quad = float(z @ w)
    tr = {k: float(np.trace(A[k])) for k in A}
    wSw = {k: float(w @ (deriv[k] @ w)) for k in A}
    score = np.array([(quad - n) / (2 * s2),
                      0.5 * (wSw["a"] - tr["a"]),
                      0.5 * (wSw["n"] - tr["n"])])
    frob, direct = {}, {}
    for ki, kj in (("a", "a"), ("a", "n"), ("n", "n")):
        frob[ki + kj] = float(trace_product_frobenius(A[ki], A[kj]))
        direct[ki + kj] = float(np.sum(A[ki] * A[kj].T))
    fisher = np.array([
        [n / (2 * s2 * s2), tr["a"] / (2 * s2), tr["n"] / (2 * s2)],
        [tr["a"] / (2 * s2), 0.5 * frob["aa"], 0.5 * frob["an"]],
        [tr["n"] / (2 * s2), 0.5 * frob["an"], 0.5 * frob["nn"]],
    ])
    return {"loglik": float(_gaussian_loglik(n, logdet, quad)), "score": score,
            "fisher": fisher, "logdet": logdet, "quad": quad,
            "trace": tr, "wSw": wSw, "trAB_frobenius": frob, "trAB_direct": direct}


def adjoint_score(locs, z, theta, sigma_nu="exact"):
    """Score of Eq. (2) in its adjoint (Frobenius) form, for the adjoint
    gradient: with w = Sigma^{-1} Z,

        dl/dtheta_i = 1/2 w^T Sigma_i w - 1/2 tr(Sigma^{-1} Sigma_i)
                    = sum_jk G_jk (Sigma_i)_jk,   G = (w w^T - Sigma^{-1}) / 2,

    written out with an explicit inverse Sigma^{-1} = cho_solve(I) and the
    entrywise sum (tr(A B) = sum_jk A_jk B_kj, B symmetric).  Also returns
    dl/dZ = -w, the gradient of Eq. (1) with respect to the observations.
    """
    theta = _check_theta(theta)
    s2 = theta[0]
    z = np.asarray(z, dtype=np.float64)
    n = z.size
    S, Sa, Sn = cov_matrices(locs, theta)
    if sigma_nu == "paper":
        Sn = _paper_sigma_nu(locs, theta)
    logdet, X = _spd_solve(S, np.hstack([z[:, None], np.eye(n)]))
    w, Sinv = X[:, 0], X[:, 1:]
    quad = float(z @ w)
    ll = _gaussian_loglik(n, logdet, quad)
    G = 0.5 * (np.outer(w, w) - Sinv)
    score = np.array([float(np.sum(G * S)) / s2, float(np.sum(G * Sa)), float(np.sum(G * Sn))])
    return {"loglik": float(ll), "score": score, "dz": -w, "quad": quad}


from .fisher_bt import (  # noqa: E402  (re-export the fit)
    OracleEvaluator,
    fisher_bt,
    l9_design,
    nelder_mead,
)
