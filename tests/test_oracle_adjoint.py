"""Pins of the oracle's adjoint form of the score (Eq. (2) written as the
Frobenius product <(w w^T - Sigma^{-1}) / 2, Sigma_i>) and of dl/dZ = -w,
against quantities that do not go through that formula:

  * Algorithm 3's route (traces of Sigma^{-1} Sigma_i by triangular solves and
    w^T Sigma_i w) on the same inputs;
  * central differences of the oracle log-likelihood in theta and in Z;
  * n = 1: dl/dsigma2 = (z^2 / sigma2 - 1) / (2 sigma2), the others 0;
  * n = 2: the bivariate closed form dl/drho composed with dC/dalpha, dC/dnu.
"""
import numpy as np
import pytest

import synth

THETAS = [(1.0, 0.1, 0.5), (1.3, 0.07, 1.2), (0.7, 0.15, 2.2), (2.0, 0.05, 0.3)]


@pytest.mark.parametrize("theta", THETAS)
def test_adjoint_equals_algorithm3(oracle_mod, theta):
    locs, z, _ = synth.dataset(250, (1.0, 0.1, 0.5), 41)
    a = oracle_mod.adjoint_score(locs, z, theta)
    e = oracle_mod.evaluate(locs, z, theta)
    n = z.size
    scale = np.array([(e["quad"] + n) / (2 * theta[0]),
                      0.5 * (abs(e["trace"]["a"]) + abs(e["wSw"]["a"])),
                      0.5 * (abs(e["trace"]["n"]) + abs(e["wSw"]["n"]))])
    assert np.all(np.abs(a["score"] - e["score"]) <= 1e-10 * scale), (a["score"], e["score"])
    assert abs(a["loglik"] - e["loglik"]) <= 1e-12 * abs(e["loglik"])


@pytest.mark.parametrize("theta", THETAS[:2])
def test_adjoint_finite_differences(oracle_mod, theta):
    locs, z, _ = synth.dataset(120, (1.0, 0.1, 0.5), 43)
    a = oracle_mod.adjoint_score(locs, z, theta)
    th = np.array(theta)
    for k in range(3):
        d = 1e-6 * th[k]
        tp, tm = th.copy(), th.copy()
        tp[k] += d
        tm[k] -= d
        fd = (oracle_mod.loglik(locs, z, tp)["loglik"] - oracle_mod.loglik(locs, z, tm)["loglik"]) / (2 * d)
        assert abs(fd - a["score"][k]) <= 1e-6 * max(1.0, abs(a["score"][k])), (k, fd, a["score"][k])
    # dl/dZ
    for k in (0, 17, 119):
        d = 1e-6
        zp, zm = z.copy(), z.copy()
        zp[k] += d
        zm[k] -= d
        fd = (oracle_mod.loglik(locs, zp, theta)["loglik"] - oracle_mod.loglik(locs, zm, theta)["loglik"]) / (2 * d)
        assert abs(fd - a["dz"][k]) <= 1e-6 * max(1.0, abs(a["dz"][k])), (k, fd, a["dz"][k])


def test_adjoint_n1(oracle_mod):
    s2, zz = 1.7, 0.9
    a = oracle_mod.adjoint_score(np.array([[0.3, 0.4]]), np.array([zz]), (s2, 0.2, 0.8))
    assert abs(a["score"][0] - (zz * zz / s2 - 1) / (2 * s2)) <= 1e-15
    assert a["score"][1] == 0.0 and a["score"][2] == 0.0
    assert abs(a["dz"][0] + zz / s2) <= 1e-15


@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.5), (1.4, 0.3, 1.7)])
def test_adjoint_n2_closed_form(oracle_mod, theta):
    locs = np.array([[0.1, 0.2], [0.16, 0.25]])
    z = np.array([0.7, -0.4])
    s2 = theta[0]
    h = np.hypot(*(locs[0] - locs[1]))
    c, ca, cn = (v[0] for v in oracle_mod.matern_entries(np.array([h]), theta))
    rho = c / s2
    D = 1 - rho * rho
    Q = z[0] ** 2 - 2 * rho * z[0] * z[1] + z[1] ** 2
    dl_drho = rho / D + (z[0] * z[1] * D - rho * Q) / (s2 * D * D)
    a = oracle_mod.adjoint_score(locs, z, theta)
    assert abs(a["score"][1] - dl_drho * ca / s2) <= 1e-12 * abs(dl_drho * ca / s2)
    assert abs(a["score"][2] - dl_drho * cn / s2) <= 1e-12 * abs(dl_drho * cn / s2)
    # sigma2: l depends on sigma2 through D * s2 and Q / s2
    dl_ds2 = -1.0 / s2 + Q / (2 * s2 * s2 * D)
    assert abs(a["score"][0] - dl_ds2) <= 1e-12 * abs(dl_ds2)
