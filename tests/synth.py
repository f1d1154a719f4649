"""Seeded synthetic inputs: locations and zero-mean Gaussian random field draws.

The one module that both sides of the parity tests read (the HIP library's
tests and benchmark, and the oracle's checks).  It lives beside the tests, not
in the product package, and imports neither the oracle nor the library.  It
holds none of the likelihood, score or Fisher arithmetic: it only *draws*
data, and the draw's covariance is evaluated with third-party routines (the
closed forms at half-integer order with numpy's exp, SciPy's Bessel K
otherwise, and numpy's LAPACK Cholesky), none of which either side uses.

Recipe (every stream is numpy Generator(PCG64(seed))):
  * uniform design: n locations iid U([0,1]^2), drawn first;
  * jittered grid: m x m cell centres (i + 1/2)/m plus independent
    U(-jitter, jitter)/m per coordinate;
  * field: w ~ N(0, I_n) drawn after the locations from the same stream,
    Z = L w with L L^T = Sigma(theta_true) the Matern covariance of Section 2.1
    (no nugget).  If Sigma(theta_true) fails the Cholesky factorisation, the
    draw is repeated with seed + 1, + 2, ... and the number of redraws is
    reported.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_locations(n: int, gen: np.random.Generator) -> np.ndarray:
    return gen.random((int(n), 2))


def jittered_grid(m: int, gen: np.random.Generator, jitter: float = 0.4) -> np.ndarray:
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    centres = np.stack([(i.ravel() + 0.5) / m, (j.ravel() + 0.5) / m], axis=1)
    return centres + gen.uniform(-jitter, jitter, size=centres.shape) / m


def _matern_for_simulation(h: np.ndarray, theta) -> np.ndarray:
    """Matern covariance used only to simulate data (library routines)."""
    from scipy.special import gamma, kv

    s2, a, nu = (float(t) for t in theta)
    x = h / a
    if nu == 0.5:
        return s2 * np.exp(-x)
    if nu == 1.5:
        return s2 * (1.0 + x) * np.exp(-x)
    if nu == 2.5:
        return s2 * (1.0 + x + x * x / 3.0) * np.exp(-x)
    out = np.full_like(x, s2)
    pos = x > 0
    xp = x[pos]
    out[pos] = s2 * (2.0 ** (1.0 - nu) / gamma(nu)) * xp ** nu * kv(nu, xp)
    return out


def grf(locs: np.ndarray, theta, gen: np.random.Generator) -> np.ndarray:
    """One realisation Z ~ N(0, Sigma(theta)); raises LinAlgError if not PD."""
    from scipy.spatial.distance import cdist

    n = locs.shape[0]
    S = np.empty((n, n))
    blk = 2048
    for r0 in range(0, n, blk):       # bounded temporaries at large n
        S[r0:r0 + blk] = _matern_for_simulation(cdist(locs[r0:r0 + blk], locs), theta)
    L = np.linalg.cholesky(S)
    del S
    w = gen.standard_normal(n)
    return L @ w


def rff_field(locs: np.ndarray, theta, gen: np.random.Generator, features: int = 4096) -> np.ndarray:
    """An approximate realisation of the Matern field by random Fourier
    features, for sizes where the exact draw (a dense host Cholesky) is out of
    reach: Z(s) = sqrt(2 sigma2 / M) sum_m cos(w_m . s + b_m) with b_m ~ U(0, 2 pi)
    and w_m from the Matern spectral density, proportional to
    (1 / alpha^2 + |w|^2)^-(nu + 1) in two dimensions, i.e. w = g / (alpha sqrt(V))
    with g ~ N(0, I_2) and V ~ chi^2 with 2 nu degrees of freedom.  Its
    covariance tends to the Matern one as M grows."""
    s2, a, nu = (float(t) for t in theta)
    g = gen.standard_normal((features, 2))
    v = gen.chisquare(2.0 * nu, features)
    w = g / (a * np.sqrt(v))[:, None]
    b = gen.uniform(0.0, 2.0 * np.pi, features)
    z = np.zeros(locs.shape[0])
    for r0 in range(0, locs.shape[0], 8192):      # bounded temporaries
        ph = locs[r0:r0 + 8192] @ w.T + b
        z[r0:r0 + 8192] = np.cos(ph).sum(axis=1)
    return np.sqrt(2.0 * s2 / features) * z


def dataset(n: int, theta_true, seed: int, design: str = "uniform", max_redraws: int = 20):
    """(locs, z, info) for a uniform or jittered-grid design."""
    for redraw in range(max_redraws + 1):
        gen = rng(seed + redraw)
        if design == "uniform":
            locs = uniform_locations(n, gen)
        elif design == "grid":
            m = int(round(np.sqrt(n)))
            if m * m != n:
                raise ValueError("grid design needs a square n")
            locs = jittered_grid(m, gen)
        else:
            raise ValueError(design)
        try:
            z = grf(locs, theta_true, gen)
        except np.linalg.LinAlgError:
            continue
        return locs, z, {"seed": seed, "redraws": redraw, "design": design,
                         "theta_true": tuple(float(t) for t in theta_true), "n": n}
    raise RuntimeError("no positive-definite draw within %d redraws" % max_redraws)


def random_thetas(k: int, seed: int, s2=(0.5, 2.0), alpha=(0.02, 0.3), nu=(0.3, 3.0)):
    """k parameter vectors drawn uniformly from a box."""
    gen = rng(seed)
    return np.stack([gen.uniform(*s2, k), gen.uniform(*alpha, k), gen.uniform(*nu, k)], axis=1)


# Named workloads (sizes of the paper's simulation settings and of the
# benchmark): n, theta_true, design, seed.
WORKLOADS = {
    # Fisher-BT from theta0 = (0.5, 0.05, 1.0) on 400 uniform points.
    "n400": dict(n=400, theta_true=(1.0, 0.1, 0.5), design="uniform", seed=1),
    # Headline evaluation size: 20,000 uniform points, theta = (1, 0.1, 0.5).
    "n20k": dict(n=20000, theta_true=(1.0, 0.1, 0.5), design="uniform", seed=20000),
    # Differentiation check: 10,000 uniform points, theta = (1, 0.1, 1.5).
    "n10k_diff": dict(n=10000, theta_true=(1.0, 0.1, 1.5), design="uniform", seed=3000),
    # Precision comparison: 50,000 uniform points, theta = (1, 0.05, 0.8); data by
    # random Fourier features (rff_field).
    "n50k": dict(n=50000, theta_true=(1.0, 0.05, 0.8), design="uniform", seed=4000),
}


def grid_workload(i_beta: int, i_nu: int):
    """The 3 x 3 jittered-grid settings on a 100 x 100 grid."""
    betas = (0.03, 0.1, 0.3)
    nus = (0.5, 1.0, 2.5)
    return dict(n=10000, theta_true=(1.0, betas[i_beta], nus[i_nu]), design="grid",
                seed=1000 + 3 * i_beta + i_nu)


def batch_workload(nf: int = 256, seed: int = 5000, n_range=(500, 4000),
                   theta_sim=(1.0, 0.1, 0.5)):
    """Many independent fields: n_f ~ U[n_range] uniform points each, data one
    realisation at theta_sim (seed seed + 1 + f), and an evaluation point
    theta_f uniform in sigma2 in [0.5, 2], alpha in [0.02, 0.3], nu in
    [0.3, 2.5].  Returns (fields [(locs, z)], thetas (nf x 3)); thetas whose
    covariance is not positive definite are redrawn by the caller with
    batch_redraw_thetas."""
    gen = rng(seed)
    ns = gen.integers(n_range[0], n_range[1] + 1, nf)
    fields = [dataset(int(n), theta_sim, seed + 1 + f)[:2] for f, n in enumerate(ns)]
    return fields, batch_redraw_thetas(np.zeros((nf, 3)), np.ones(nf, bool), gen)


def batch_fit_workload(nf: int = 256, seed: int = 6000, n_range=(500, 4000), approx=None,
                       progress=None, draw: str = "exact"):
    """Replicate fields for batched fits: n_f ~ U[n_range] uniform points
    each, a true theta_f uniform in sigma2 in [0.5, 2], alpha in [0.02, 0.3],
    nu in [0.3, 2.5], and one realisation at theta_f (seed seed + 1 + f):
    the exact draw (draw="exact"; where Sigma(theta_f) is numerically
    indefinite it is replaced by the random-Fourier-feature draw on the same
    locations, and f is appended to `approx` when given), or the
    random-Fourier-feature draw for every field (draw="rff": the exact draw
    costs a dense host Cholesky and n^2 Bessel values per field).
    Returns (fields [(locs, z)], true thetas (nf x 3))."""
    gen = rng(seed)
    ns = gen.integers(n_range[0], n_range[1] + 1, nf)
    thetas = batch_redraw_thetas(np.zeros((nf, 3)), np.ones(nf, bool), gen)
    fields = []
    for f, n in enumerate(ns):
        try:
            if draw != "exact":
                raise RuntimeError("approximate draw requested")
            fields.append(dataset(int(n), tuple(thetas[f]), seed + 1 + f, max_redraws=0)[:2])
        except RuntimeError:
            g = rng(seed + 1 + f)
            locs = uniform_locations(int(n), g)
            fields.append((locs, rff_field(locs, thetas[f], g)))
            if approx is not None:
                approx.append(f)
        if progress is not None:
            progress(f)
    return fields, thetas


def batch_redraw_thetas(thetas, which, gen):
    """Redraw the evaluation points of the fields flagged in `which`."""
    thetas = np.array(thetas, dtype=np.float64)
    for f in np.flatnonzero(which):
        thetas[f] = (gen.uniform(0.5, 2.0), gen.uniform(0.02, 0.3), gen.uniform(0.3, 2.5))
    return thetas
