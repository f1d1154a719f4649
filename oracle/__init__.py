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
  __init__.py      Algorithms 2 and 3 written step by step with LAPACK primitives
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
# Algorithm 2: log-likelihood; Algorithm 3: log-likelihood, score, Fisher
# --------------------------------------------------------------------------
def _check_theta(theta):
    theta = np.asarray(theta, dtype=np.float64)
    if theta.shape != (3,) or not np.all(np.isfinite(theta)) or np.any(theta <= 0):
        raise ValueError("theta must be three finite positive numbers (sigma2, alpha, nu)")
    return theta


def _cholesky(S):
    try:
        return np.linalg.cholesky(S)
    except np.linalg.LinAlgError as e:
        raise NotPositiveDefinite(str(e)) from None


def trace_product_frobenius(A, B):
    """trace(AB) via the Frobenius identity of Eq. (5)."""
    return 0.5 * (np.sum((A + B.T) ** 2) - np.sum(A ** 2) - np.sum(B ** 2))


def loglik(locs, z, theta):
    """Algorithm 2.  Returns dict(loglik, logdet, quad)."""
    theta = _check_theta(theta)
    z = np.asarray(z, dtype=np.float64)
    n = z.size
    (S,) = cov_matrices(locs, theta, which=("S",))            # Sigma(theta)
    L = _cholesky(S)                                          # Sigma = L L^T
    logdet = 2.0 * np.sum(np.log(np.diag(L)))                 # 2 sum log l_ii
    Y = scipy.linalg.solve_triangular(L, z, lower=True)       # Y = L^{-1} Z
    quad = float(Y @ Y)                                       # Z^T Sigma^{-1} Z = Y^T Y
    ll = -0.5 * n * np.log(2 * np.pi) - 0.5 * logdet - 0.5 * quad   # Eq. (1)
    return {"loglik": float(ll), "logdet": float(logdet), "quad": quad}


def _paper_sigma_nu(locs, theta):
    """Dense Sigma_nu by the paper's case scheme (oracle.paper_mode)."""
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


def evaluate(locs, z, theta, sigma_nu="exact"):
    """Algorithm 3: log-likelihood, score (Eq. 2) and Fisher information (Eq. 3).

    The score is over theta = (sigma2, alpha, nu).  Besides the results it
    returns the intermediate traces, and every Fisher entry of the alpha/nu
    block both by the Frobenius identity of Eq. (5) and by the direct sum
    sum_jk A_jk B_kj.
    """
    theta = _check_theta(theta)
    s2 = theta[0]
    z = np.asarray(z, dtype=np.float64)
    n = z.size
    S, Sa, Sn = cov_matrices(locs, theta)
    if sigma_nu == "paper":
        Sn = _paper_sigma_nu(locs, theta)
    # Step 1: log-likelihood
    L = _cholesky(S)
    logdet = 2.0 * np.sum(np.log(np.diag(L)))
    Y = scipy.linalg.solve_triangular(L, z, lower=True)
    quad = float(Y @ Y)
    ll = -0.5 * n * np.log(2 * np.pi) - 0.5 * logdet - 0.5 * quad
    # Step 2: sigma2 entries
    score = np.zeros(3)
    fisher = np.zeros((3, 3))
    score[0] = (quad - n) / (2 * s2)
    fisher[0, 0] = n / (2 * s2 ** 2)
    # Steps 3 and 4: alpha and nu
    w = scipy.linalg.cho_solve((L, True), z)                  # w = Sigma^{-1} Z
    A = {}
    tr, wv = {}, {}
    for idx, (key, Si) in ((1, ("a", Sa)), (2, ("n", Sn))):
        Ai = scipy.linalg.cho_solve((L, True), Si)            # A = Sigma^{-1} Sigma_i
        A[key] = Ai
        tr[key] = float(np.trace(Ai))
        v = Si @ w                                            # v = Sigma_i Sigma^{-1} Z
        wv[key] = float(w @ v)
        fisher[0, idx] = fisher[idx, 0] = tr[key] / (2 * s2)
        score[idx] = -0.5 * tr[key] + 0.5 * wv[key]           # Eq. (2)
    frob, direct = {}, {}
    for (i, ki), (j, kj) in (((1, "a"), (1, "a")), ((1, "a"), (2, "n")), ((2, "n"), (2, "n"))):
        frob[ki + kj] = trace_product_frobenius(A[ki], A[kj])
        direct[ki + kj] = float(np.sum(A[ki] * A[kj].T))
        fisher[i, j] = fisher[j, i] = 0.5 * frob[ki + kj]     # Eq. (3) via Eq. (5)
    return {"loglik": float(ll), "score": score, "fisher": fisher,
            "logdet": float(logdet), "quad": quad,
            "trace": tr, "wSw": wv, "trAB_frobenius": frob, "trAB_direct": direct}


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
    L = _cholesky(S)
    logdet = 2.0 * np.sum(np.log(np.diag(L)))
    w = scipy.linalg.cho_solve((L, True), z)
    quad = float(z @ w)
    ll = -0.5 * n * np.log(2 * np.pi) - 0.5 * logdet - 0.5 * quad
    Sinv = scipy.linalg.cho_solve((L, True), np.eye(n))
    G = 0.5 * (np.outer(w, w) - Sinv)
    score = np.array([float(np.sum(G * S)) / s2, float(np.sum(G * Sa)), float(np.sum(G * Sn))])
    return {"loglik": float(ll), "score": score, "dz": -w, "quad": quad}


from .fisher_bt import (  # noqa: E402  (re-export the fit)
    OracleEvaluator,
    fisher_bt,
    l9_design,
    nelder_mead,
)
