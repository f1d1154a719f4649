"""GPU paper mode (Sigma_nu by the case scheme of Supplementary A) against
the oracle's paper mode on the same inputs.

Both sides evaluate the same truncated series / expansions / differences in
FP64 but in a different order, so they agree only to the scheme's own
rounding sensitivity: entries to 2e-6 relative plus 2e-6 of C (the central
difference amplifies the quadratures' rounding by 1 / lag), with nu kept
>= 0.2 from the integers where the series' cancellation is mild, plus nu = 1
and nu = 1/2, where the central difference replaces the series (x < 8.5) or
the Hankel expansion (x >= 30).  Score and Fisher are then compared at the
tolerances that entry-level agreement supports (1e-6 of the per-term score
scale and of sqrt(I_ii I_jj); 1e-5 where the central difference is used).  The mode is active (the paper-mode Sigma_nu
differs from the exact one), the log-likelihood is the same bit for bit, and
the sigma2 and alpha score components are unchanged by it.
"""
import sys

import numpy as np
import pytest

import paper_2601_11437_amd as fbt
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = fbt.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.3), (1.3, 0.05, 0.7), (0.8, 0.02, 1.3),
                                   (1.1, 0.03, 2.2), (1.0, 0.1, 1.0), (0.9, 0.01, 0.5)])
def test_paper_sigma_nu_entries(ctx, oracle_mod, theta):
    say("paper entries theta=%s" % (theta,))
    n = 300
    locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 17)
    ctx.set_data(locs, z)
    ctx.set_sigma_nu_mode(fbt.SIGMA_NU_PAPER)
    try:
        G = ctx.covariance(theta, 2)
    finally:
        ctx.set_sigma_nu_mode(fbt.SIGMA_NU_EXACT)
    R = oracle_mod._paper_sigma_nu(locs, theta)
    (S,) = oracle_mod.cov_matrices(locs, theta, which=("S",))
    # the central difference (lag 1e-9) turns a 1e-15 relative difference of
    # the two quadratures of x^nu K_nu into ~5e-7 of C in dC/dnu
    tol = 2e-6 * np.abs(R) + 2e-6 * S + 1e-14 * theta[0]
    assert np.all(np.abs(G - R) <= tol), np.max(np.abs(G - R) / tol)
    E = ctx.covariance(theta, 2)
    assert not np.array_equal(E, G)


@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.7), (1.2, 0.05, 1.3), (1.0, 0.1, 1.0)])
def test_paper_mode_eval(ctx, oracle_mod, theta):
    say("paper eval theta=%s" % (theta,))
    n = 400
    locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 1)
    ctx.set_data(locs, z)
    want = oracle_mod.evaluate(locs, z, theta, sigma_nu="paper")
    ll_e, sc_e, fi_e = ctx.eval(theta)
    ctx.set_sigma_nu_mode(fbt.SIGMA_NU_PAPER)
    try:
        ll, sc, fi = ctx.eval(theta)
        llg, scg = ctx.grad(theta)
    finally:
        ctx.set_sigma_nu_mode(fbt.SIGMA_NU_EXACT)
    assert ll == ll_e == llg
    # where the central difference (lag 1e-9) replaces the series, each side's
    # dC/dnu carries its own ~1e-7 C rounding noise; the sums then agree to ~1e-6
    fd = abs(theta[2] - round(theta[2])) <= 1e-6 or abs(theta[2] + 0.5 - round(theta[2] + 0.5)) <= 1e-6
    tol = 1e-5 if fd else 1e-6
    scale = np.array([(want["quad"] + n) / (2 * theta[0]),
                      0.5 * (abs(want["trace"]["a"]) + abs(want["wSw"]["a"])),
                      0.5 * (abs(want["trace"]["n"]) + abs(want["wSw"]["n"]))])
    assert np.all(np.abs(sc - want["score"]) <= tol * scale), (sc, want["score"])
    assert np.all(np.abs(scg - want["score"]) <= tol * scale), (scg, want["score"])
    d = np.sqrt(np.outer(np.diag(want["fisher"]), np.diag(want["fisher"])))
    assert np.all(np.abs(fi - want["fisher"]) <= tol * d)
    assert sc[0] == sc_e[0] and sc[1] == sc_e[1]
    say("paper - exact nu score: %.3e (scale %.3e)" % (sc[2] - sc_e[2], scale[2]))


@pytest.mark.parametrize("theta_true", [(1.0, 0.1, 1.0), (1.0, 0.1, 0.7)])
def test_paper_mode_fit_shift(ctx, theta_true):
    """How far the paper's scheme for Sigma_nu moves the Fisher-BT estimate:
    the same fit (L9 start within the paper's bounds) in both modes on 2,000
    uniform points.  Both must converge; the shift of theta-hat is printed and
    must stay far below the estimate's own standard error (checked at 1e-3
    relative)."""
    locs, z, _ = synth.dataset(2000, theta_true, 7)
    ctx.set_data(locs, z)
    lo, hi = (0.01, 0.01, 0.01), (5.0, 5.0, 2.0)
    exact = ctx.fit(lo=lo, hi=hi)
    ctx.set_sigma_nu_mode(fbt.SIGMA_NU_PAPER)
    try:
        paper = ctx.fit(lo=lo, hi=hi)
    finally:
        ctx.set_sigma_nu_mode(fbt.SIGMA_NU_EXACT)
    rel = np.abs(paper["theta"] - exact["theta"]) / np.abs(exact["theta"])
    say("theta_true %s: exact %s (%d iters, NM %d)  paper %s (%d iters, NM %d)  rel shift %s"
        % (theta_true, np.round(exact["theta"], 6), exact["n_iter"], exact["used_nelder_mead"],
           np.round(paper["theta"], 6), paper["n_iter"], paper["used_nelder_mead"], rel))
    assert exact["converged"] and paper["converged"]
    assert np.all(rel <= 1e-3)
