"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.

Tolerances (FP64 throughout):
  * log-likelihood (Eq. 1): |d l| <= 1e-10 |l|;
  * score (Eq. 2), per term: |d l_i| <= 1e-10 * (|tr(Sigma^-1 Sigma_i)| + |w' Sigma_i w|) / 2
    (for sigma2 the terms are (Z' Sigma^-1 Z + n) / (2 sigma2)), because the score
    is a difference of two such terms and vanishes at the optimum;
  * Fisher (Eq. 3): |d I_ij| <= 1e-8 sqrt(I_ii I_jj);
  * covariance entries: |d C| <= 1e-13 |C| + 1e-300; the derivatives add a
    cancellation allowance 1e-14 |C| (1 + |log x| + |psi(nu)|) for C_nu (two
    terms of that size cancel as x -> 0) and 1e-14 |C| for C_alpha.
Gates apply where eps * cond(Sigma) <= 1e-6 (conditioning is checked).
"""
import math
import sys

import numpy as np
import pytest
import scipy.special as sp

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


THETAS = [(1.0, 0.1, 0.5), (0.6, 0.05, 1.4), (2.0, 0.2, 0.25), (1.5, 0.07, 1.0),
          (0.8, 0.3, 0.05), (1.2, 0.02, 2.6)]


def _dist(locs):
    d = locs[:, None, :] - locs[None, :, :]
    return np.sqrt((d ** 2).sum(-1))


@pytest.mark.parametrize("n", [1, 2, 63, 255, 256, 257, 700])
@pytest.mark.parametrize("theta", THETAS)
def test_covariance_entries(ctx, oracle_mod, n, theta):
    say("covariance n=%d theta=%s" % (n, theta))
    locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 100 + n)
    ctx.set_data(locs, z)
    S, Sa, Sn = oracle_mod.cov_matrices(locs, theta)
    G = [ctx.covariance(theta, w) for w in (0, 1, 2)]
    x = _dist(locs) / theta[1]
    with np.errstate(divide="ignore"):
        lx = np.where(x > 0, np.abs(np.log(np.where(x > 0, x, 1.0))), 0.0)
    base = 1e-13 * np.abs(S) + 1e-300
    assert np.all(np.abs(G[0] - S) <= base), np.max(np.abs(G[0] - S) / (np.abs(S) + 1e-300))
    assert np.all(np.abs(G[1] - Sa) <= 1e-13 * np.abs(Sa) + 1e-14 * np.abs(S) + 1e-300)
    tol_n = 1e-13 * np.abs(Sn) + 1e-14 * np.abs(S) * (1 + lx + abs(sp.digamma(theta[2]))) + 1e-300
    assert np.all(np.abs(G[2] - Sn) <= tol_n), np.max(np.abs(G[2] - Sn) / tol_n)
    np.testing.assert_array_equal(G[0], G[0].T)
    np.testing.assert_array_equal(G[1], G[1].T)
    np.testing.assert_array_equal(G[2], G[2].T)


def _cond(locs, theta, oracle_mod):
    (S,) = oracle_mod.cov_matrices(locs, theta, which=("S",))
    w = np.linalg.eigvalsh(S)
    return w[-1] / w[0] if w[0] > 0 else math.inf


CASES = [(1, THETAS[0]), (2, THETAS[1]), (100, THETAS[2]), (255, THETAS[0]), (256, THETAS[3]),
         (257, THETAS[4]), (600, THETAS[0]), (600, THETAS[1]), (600, THETAS[5]),
         (1500, THETAS[0]), (1500, THETAS[3])]


WPHASES = [fbt.WPHASE_TWO_SIDED, fbt.WPHASE_SOLVES]


@pytest.mark.parametrize("wphase", WPHASES, ids=["two_sided", "solves"])
@pytest.mark.parametrize("n,theta", CASES + [(3000, THETAS[0]), (3000, THETAS[3])])
def test_eval_parity(ctx, oracle_mod, n, theta, wphase):
    say("eval n=%d theta=%s wphase=%d" % (n, theta, wphase))
    locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 1000 + n)
    if n > 2:
        kappa = _cond(locs, theta, oracle_mod)
        assert np.finfo(float).eps * kappa <= 1e-6, kappa
    ctx.set_data(locs, z)
    ctx.set_wphase(wphase)
    try:
        _eval_parity(ctx, oracle_mod, locs, z, n, theta)
    finally:
        ctx.set_wphase(fbt.WPHASE_TWO_SIDED)


def _eval_parity(ctx, oracle_mod, locs, z, n, theta):
    want = oracle_mod.evaluate(locs, z, theta)
    ll = ctx.loglik(theta)
    assert abs(ll - want["loglik"]) <= 1e-10 * abs(want["loglik"])
    gll, score, fisher = ctx.eval(theta)
    assert abs(gll - want["loglik"]) <= 1e-10 * abs(want["loglik"])
    scale = np.array([(want["quad"] + n) / (2 * theta[0]),
                      0.5 * (abs(want["trace"]["a"]) + abs(want["wSw"]["a"])),
                      0.5 * (abs(want["trace"]["n"]) + abs(want["wSw"]["n"]))])
    assert np.all(np.abs(score - want["score"]) <= 1e-10 * scale), (score, want["score"], scale)
    I = want["fisher"]
    d = np.sqrt(np.outer(np.diag(I), np.diag(I)))
    assert np.all(np.abs(fisher - I) <= 1e-8 * d), (fisher, I)
    t = ctx.eval_terms(theta)
    ref = [want["logdet"], want["quad"], want["trace"]["a"], want["trace"]["n"], want["wSw"]["a"],
           want["wSw"]["n"], want["trAB_direct"]["aa"], want["trAB_direct"]["an"],
           want["trAB_direct"]["nn"]]
    sc = [abs(want["logdet"]) + n, want["quad"], scale[1], scale[2], scale[1], scale[2],
          I[1, 1] * 2, d[1, 2] * 2, I[2, 2] * 2]
    for k in range(9):
        assert abs(t[k] - ref[k]) <= 1e-9 * sc[k] + 1e-300, (k, t[k], ref[k])


@pytest.mark.parametrize("n", [300, 700])
def test_factor_parity(ctx, oracle_mod, n):
    say("factor n=%d" % n)
    locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 2000 + n)
    theta = (1.0, 0.1, 0.5)
    ctx.set_data(locs, z)
    L = ctx.factor(theta)
    (S,) = oracle_mod.cov_matrices(locs, theta, which=("S",))
    Lref = np.linalg.cholesky(S)
    assert np.max(np.abs(L - Lref)) <= 1e-12 * np.max(np.abs(Lref))
    np.testing.assert_array_equal(np.triu(L, 1), 0.0)


def test_determinism(ctx):
    say("determinism")
    locs, z, _ = synth.dataset(900, (1.0, 0.1, 0.5), 5)
    ctx.set_data(locs, z)
    a = ctx.eval_terms((1.1, 0.09, 0.7))
    b = ctx.eval_terms((1.1, 0.09, 0.7))
    np.testing.assert_array_equal(a, b)
    # eval right after loglik at the same theta reuses the factor: same numbers
    ctx.loglik((1.1, 0.09, 0.7))
    c = ctx.eval_terms((1.1, 0.09, 0.7))
    np.testing.assert_array_equal(a, c)


def test_factorisation_repeats_bitwise(ctx):
    """Sixty factorisations of one covariance give the bitwise same
    log-likelihood and factor: every reduction has a fixed order and no
    workgroup reads a value another one may still be writing (a regression
    test for an in-place race in the diagonal-block kernel, seen in about one
    launch in fifty)."""
    say("factorisation repeats")
    locs, z, _ = synth.dataset(1000, (1.0, 0.1, 0.5), 6)
    ctx.set_data(locs, z)
    theta = (0.9, 0.07, 1.3)
    ref = ctx.factor(theta)
    lls = {ctx.loglik(theta) for _ in range(60)}
    assert len(lls) == 1
    np.testing.assert_array_equal(ctx.factor(theta), ref)


def test_not_positive_definite(ctx, oracle_mod):
    """A covariance that is numerically indefinite (range 50 and smoothness 4
    on 300 points of the unit square: condition number far beyond 1/eps) fails
    the factorisation: LAPACK in the oracle and the GPU both report it."""
    say("notpd")
    locs, z, _ = synth.dataset(300, (1.0, 0.1, 0.5), 6)
    theta = (1.0, 50.0, 4.0)
    with pytest.raises(oracle_mod.NotPositiveDefinite):
        oracle_mod.loglik(locs, z, theta)
    ctx.set_data(locs, z)
    with pytest.raises(fbt.FisherBTError) as e:
        ctx.loglik(theta)
    assert e.value.status == fbt.ENOTPD and 0 < e.value.pivot < 300
    with pytest.raises(fbt.FisherBTError) as e:
        ctx.eval(theta)
    assert e.value.status == fbt.ENOTPD
    # the context stays usable
    ok = oracle_mod.loglik(locs, z, (1.0, 0.1, 0.5))["loglik"]
    assert abs(ctx.loglik((1.0, 0.1, 0.5)) - ok) <= 1e-10 * abs(ok)


def test_invalid_arguments(ctx):
    say("invalid")
    locs, z, _ = synth.dataset(50, (1.0, 0.1, 0.5), 7)
    ctx.set_data(locs, z)
    for bad in ((0.0, 0.1, 0.5), (1.0, -0.1, 0.5), (1.0, 0.1, float("nan"))):
        with pytest.raises(fbt.FisherBTError) as e:
            ctx.loglik(bad)
        assert e.value.status == fbt.EINVAL
    bad_z = z.copy()
    bad_z[3] = np.inf
    with pytest.raises(fbt.FisherBTError) as e:
        ctx.set_data(locs, bad_z)
    assert e.value.status == fbt.EINVAL


def test_device_pointer_input(ctx, oracle_mod):
    say("device input")
    torch = pytest.importorskip("torch")
    locs, z, _ = synth.dataset(400, (1.0, 0.1, 0.5), 8)
    ctx.set_data(torch.tensor(locs, device="cuda"), torch.tensor(z, device="cuda"))
    want = oracle_mod.loglik(locs, z, (1.0, 0.1, 0.5))["loglik"]
    assert abs(ctx.loglik((1.0, 0.1, 0.5)) - want) <= 1e-10 * abs(want)


def test_fit_n400_matches_oracle(ctx, oracle_mod):
    """Fisher-BT from theta0 = (0.5, 0.05, 1.0), at most 50 iterations, on 400
    uniform points with theta_true = (1, 0.1, 0.5)."""
    say("fit n400")
    w = synth.WORKLOADS["n400"]
    locs, z, _ = synth.dataset(w["n"], w["theta_true"], w["seed"])
    ctx.set_data(locs, z)
    it_gpu = []
    got = ctx.fit(theta0=(0.5, 0.05, 1.0), max_iter=50,
                  callback=lambda it, th, ll, g, f: it_gpu.append((th, ll, g, f)))
    want = oracle_mod.fisher_bt(oracle_mod.OracleEvaluator(locs, z), theta0=(0.5, 0.05, 1.0),
                                max_iter=50)
    say("gpu", got["theta"], got["n_iter"], "oracle", want["theta"], want["n_iter"])
    assert got["converged"] and want["converged"]
    assert (got["n_loglik_calls"], got["n_grad_calls"]) == (want["n_loglik_calls"], want["n_grad_calls"])
    np.testing.assert_allclose(got["theta"], want["theta"], rtol=1e-6)
    assert len(it_gpu) == got["n_iter"] + 1


def test_fit_l9_n1500_matches_oracle(ctx, oracle_mod):
    """Fisher-BT from the L9 start (Table 1, the paper's bounds) on 1,500
    uniform points: the same path as the oracle's driver on the oracle's
    evaluations (call counts, convergence) and theta-hat to 1e-6 relative."""
    say("fit n1500 L9")
    locs, z, _ = synth.dataset(1500, (1.0, 0.1, 0.5), 2025)
    ctx.set_data(locs, z)
    got = ctx.fit()
    want = oracle_mod.fisher_bt(oracle_mod.OracleEvaluator(locs, z))
    say("gpu", got["theta"], got["n_loglik_calls"], got["n_grad_calls"], "oracle", want["theta"],
        want["n_loglik_calls"], want["n_grad_calls"])
    assert got["converged"] and want["converged"]
    assert got["used_nelder_mead"] == want["used_nelder_mead"]
    assert (got["n_loglik_calls"], got["n_grad_calls"]) == (want["n_loglik_calls"], want["n_grad_calls"])
    np.testing.assert_allclose(got["theta"], want["theta"], rtol=1e-6)


@pytest.mark.parametrize("n,theta", [(600, (1.0, 0.1, 0.5)), (1500, (1.5, 0.07, 1.0))])
def test_mixed_precision(ctx, oracle_mod, n, theta):
    """Mixed form: the trace-phase updates on FP32 MFMA.  The log-likelihood is
    the FP64 one bit for bit; score and Fisher carry FP32 rounding of the two
    block solves: per-term score error <= 1e-5 and Fisher <= 1e-4 relative on
    these moderately conditioned cases (measured 4e-8 .. 5e-6 and 3e-8 .. 7e-7)."""
    say("mixed n=%d theta=%s" % (n, theta))
    locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 3000 + n)
    ctx.set_data(locs, z)
    want = oracle_mod.evaluate(locs, z, theta)
    ll64, s64, f64 = ctx.eval(theta)
    ctx.set_precision(fbt.MIXED_FP32)
    try:
        ll, score, fisher = ctx.eval(theta)
        ll_only = ctx.loglik(theta)
    finally:
        ctx.set_precision(fbt.FP64)
    assert ll == ll64 and ll_only == ll64
    scale = np.array([(want["quad"] + n) / (2 * theta[0]),
                      0.5 * (abs(want["trace"]["a"]) + abs(want["wSw"]["a"])),
                      0.5 * (abs(want["trace"]["n"]) + abs(want["wSw"]["n"]))])
    assert np.all(np.abs(score - want["score"]) <= 1e-5 * scale)
    d = np.sqrt(np.outer(np.diag(want["fisher"]), np.diag(want["fisher"])))
    assert np.all(np.abs(fisher - want["fisher"]) <= 1e-4 * d)
    assert np.array_equal(score[:1], s64[:1])          # sigma2 score: FP64 quadratic form


@pytest.mark.parametrize("n,theta", [(600, (1.0, 0.1, 0.5)), (1500, (1.5, 0.07, 1.0))])
def test_mixed_bf16(ctx, oracle_mod, n, theta):
    """BF16 operands with FP32 sums in the trace-phase updates: the
    log-likelihood is the FP64 one bit for bit, the sigma2 score too; the other
    score terms and the Fisher entries carry bfloat16 rounding (eps = 2^-8) of
    the W phase's updates: measured against the oracle on MI355X (two-sided
    W phase) 1.8e-5 .. 3.2e-3 of the per-term scale and 3.3e-4 .. 2.0e-2
    relative in Fisher; the gates are 5e-2."""
    say("bf16 n=%d theta=%s" % (n, theta))
    locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 3000 + n)
    ctx.set_data(locs, z)
    want = oracle_mod.evaluate(locs, z, theta)
    ll64, s64, f64 = ctx.eval(theta)
    ctx.set_precision(fbt.MIXED_BF16)
    try:
        ll, score, fisher = ctx.eval(theta)
    finally:
        ctx.set_precision(fbt.FP64)
    assert ll == ll64 and score[0] == s64[0]
    scale = np.array([(want["quad"] + n) / (2 * theta[0]),
                      0.5 * (abs(want["trace"]["a"]) + abs(want["wSw"]["a"])),
                      0.5 * (abs(want["trace"]["n"]) + abs(want["wSw"]["n"]))])
    err = np.abs(score - want["score"]) / scale
    I = want["fisher"]
    d = np.sqrt(np.outer(np.diag(I), np.diag(I)))
    say("against the oracle: score err / scale", err, "fisher rel", np.max(np.abs(fisher - I) / d))
    assert abs(ll - want["loglik"]) <= 1e-10 * abs(want["loglik"])
    assert np.all(err <= 5e-2) and np.all(np.abs(fisher - I) <= 5e-2 * d)
    assert np.any(np.abs(score - s64)[1:] > 0)          # the BF16 path really ran


@pytest.mark.parametrize("n,theta", [(600, (1.0, 0.1, 0.5)), (1500, (1.5, 0.07, 1.0))])
def test_mixed_fp32_all(ctx, oracle_mod, n, theta):
    """FBT_MIXED_FP32_ALL: the Cholesky trailing updates in FP32 as well, so
    every term carries FP32 rounding of the factor; against the oracle
    (measured on MI355X, no refinement, the default): loglik 1.9e-8 / 1.3e-5
    relative, score 1.1e-7 / 3.0e-5 of its per-term scale, Fisher 1.2e-6 /
    3.0e-6 relative at n = 600 / 1,500 (with two refinement steps: loglik
    1.1e-7 / 2.6e-7, score 1.6e-7 / 7.0e-8, see test_fp32_all_refinement).
    Gates: loglik 1e-4, score 3e-4, Fisher 1e-4.  A fit refuses the form."""
    say("fp32-all n=%d theta=%s" % (n, theta))
    locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 3000 + n)
    ctx.set_data(locs, z)
    want = oracle_mod.evaluate(locs, z, theta)
    ctx.set_precision(fbt.MIXED_FP32_ALL)
    try:
        ll, score, fisher = ctx.eval(theta)
        ll_only = ctx.loglik(theta)
        with pytest.raises(fbt.FisherBTError) as e:
            ctx.fit()
        assert e.value.status == fbt.EINVAL
    finally:
        ctx.set_precision(fbt.FP64)
    scale = np.array([(want["quad"] + n) / (2 * theta[0]),
                      0.5 * (abs(want["trace"]["a"]) + abs(want["wSw"]["a"])),
                      0.5 * (abs(want["trace"]["n"]) + abs(want["wSw"]["n"]))])
    e_ll = abs(ll - want["loglik"]) / abs(want["loglik"])
    err = np.abs(score - want["score"]) / scale
    I = want["fisher"]
    d = np.sqrt(np.outer(np.diag(I), np.diag(I)))
    e_f = np.max(np.abs(fisher - I) / d)
    say("against the oracle: loglik %.2e score/scale %s fisher %.2e" % (e_ll, err, e_f))
    assert ll_only == ll
    assert e_ll <= 1e-4 and np.all(err <= 3e-4) and e_f <= 1e-4
    assert e_ll > 0                                     # the FP32 factorisation really ran


@pytest.mark.parametrize("n,theta", [(600, (1.0, 0.02, 0.5)), (1500, (1.2, 0.015, 0.8))])
def test_mixed_bf16_all(ctx, oracle_mod, n, theta):
    """FBT_MIXED_BF16_ALL: the Cholesky trailing updates with bfloat16
    operands and FP32 sums too, on short-range (well-conditioned) covariances,
    against the oracle.  Measured on MI355X at n = 600 / 1,500: loglik
    5.5e-5 / 1.4e-5 relative, score up to 5.9e-4 / 1.2e-3 of its per-term
    scale, Fisher 4.5e-3 / 1.4e-2 relative; the quadratic forms q and u_i
    1e-4 / 0.13 unrefined, and after 2, 4, 8 refinement steps of w 6e-7,
    7e-10, 7e-16 / 2.4e-3, 2.6e-4, 2.0e-7 (the log determinant and the
    traces keep the factor's bfloat16 rounding).  Gates: loglik 1e-2, score
    1e-1, Fisher 1e-1; refinement: two steps gain at least 20 times, more
    steps never lose, eight reach 1e-6."""
    say("bf16-all n=%d theta=%s" % (n, theta))
    locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 3000 + n)
    ctx.set_data(locs, z)
    want = oracle_mod.evaluate(locs, z, theta)
    ctx.set_precision(fbt.MIXED_BF16_ALL)
    try:
        ll, score, fisher = ctx.eval(theta)
        t0 = ctx.eval_terms(theta)
        tr = {}
        for k in (2, 4, 8):
            ctx.set_refinement(k)
            tr[k] = ctx.eval_terms(theta)
        with pytest.raises(fbt.FisherBTError) as e:
            ctx.fit()
        assert e.value.status == fbt.EINVAL
    finally:
        ctx.set_refinement(0)
        ctx.set_precision(fbt.FP64)
    scale = np.array([(want["quad"] + n) / (2 * theta[0]),
                      0.5 * (abs(want["trace"]["a"]) + abs(want["wSw"]["a"])),
                      0.5 * (abs(want["trace"]["n"]) + abs(want["wSw"]["n"]))])
    e_ll = abs(ll - want["loglik"]) / abs(want["loglik"])
    err = np.abs(score - want["score"]) / scale
    I = want["fisher"]
    d = np.sqrt(np.outer(np.diag(I), np.diag(I)))
    e_f = np.max(np.abs(fisher - I) / d)
    ref = np.array([want["quad"], want["wSw"]["a"], want["wSw"]["n"]])
    q0 = np.abs(np.array([t0[1], t0[4], t0[5]]) - ref) / np.abs(ref)
    qk = {k: np.abs(np.array([t[1], t[4], t[5]]) - ref) / np.abs(ref) for k, t in tr.items()}
    say("against the oracle: loglik %.2e score/scale %s fisher %.2e; quadratic forms "
        "unrefined %s, after 2/4/8 refinement steps %s %s %s"
        % (e_ll, err, e_f, q0, qk[2], qk[4], qk[8]))
    assert e_ll > 0                                     # the BF16 factorisation really ran
    assert e_ll <= 1e-2 and np.all(err <= 1e-1) and e_f <= 1e-1
    # refinement converges
    assert np.all(qk[2] <= 0.05 * q0)
    assert np.all(qk[8] <= np.maximum(qk[4], 1e-13)) and np.all(qk[4] <= np.maximum(qk[2], 1e-13))
    assert np.all(qk[8] <= 1e-6)
    for k in (2, 4, 8):                                 # log det and traces untouched
        assert tr[k][0] == t0[0] and tr[k][2] == t0[2] and tr[k][3] == t0[3]


@pytest.mark.parametrize("n,theta", [(2, (1.0, 0.1, 0.5)), (257, (0.8, 0.12, 0.9)),
                                     (600, (1.0, 0.1, 0.5)), (1500, (1.5, 0.07, 1.0))])
def test_fp32_all_refinement(ctx, oracle_mod, n, theta):
    """FBT_MIXED_FP32_ALL with iterative refinement of w = Sigma^{-1} Z (the
    residual in FP64 from a copy of Sigma, corrections from the FP32-updated
    factor): the quadratic forms q = Z^T Sigma^{-1} Z and u_i = w^T Sigma_i w
    against the oracle, without refinement (the default) and after two steps.
    Refinement leaves log det and the traces untouched (bitwise) and brings q
    and u_i to FP64 accuracy (gate 1e-10 relative, and at least 100 times
    below the unrefined error).  Measured on MI355X: unrefined 2.3e-7 - 5.0e-7
    (n = 600) and 1.0e-5 - 3.7e-5 (n = 1,500), refined 8e-16 - 3.1e-15 and
    2.2e-11 - 7.3e-11.  The log-likelihood and score assembled from either
    set of terms are reported: refinement removes the quadratic forms' share
    of the error but not log det's and the traces', with which it partly
    cancels, so they need not get closer to the oracle."""
    say("fp32-all refinement n=%d theta=%s" % (n, theta))
    locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 3000 + n)
    ctx.set_data(locs, z)
    want = oracle_mod.evaluate(locs, z, theta)
    ctx.set_precision(fbt.MIXED_FP32_ALL)
    try:
        with pytest.raises(fbt.FisherBTError) as e:
            ctx.set_refinement(17)
        assert e.value.status == fbt.EINVAL
        ctx.set_refinement(0)
        t0 = ctx.eval_terms(theta)
        ctx.set_refinement(2)
        t2 = ctx.eval_terms(theta)
        ll2 = ctx.loglik(theta)
    finally:
        ctx.set_refinement(0)
        ctx.set_precision(fbt.FP64)
    ref = np.array([want["quad"], want["wSw"]["a"], want["wSw"]["n"]])
    # the log-likelihood and score from each set of terms, against the oracle
    # (reported: whether refinement brings them closer depends on theta)
    for tag, t in (("unrefined", t0), ("refined", t2)):
        ll_t = -0.5 * n * np.log(2 * np.pi) - 0.5 * t[0] - 0.5 * t[1]
        sc_t = np.array([(t[1] - n) / (2 * theta[0]), 0.5 * (t[4] - t[2]), 0.5 * (t[5] - t[3])])
        scale = np.array([(want["quad"] + n) / (2 * theta[0]),
                          0.5 * (abs(want["trace"]["a"]) + abs(want["wSw"]["a"])),
                          0.5 * (abs(want["trace"]["n"]) + abs(want["wSw"]["n"]))])
        say("%s: loglik %.2e score/scale %s" % (tag, abs(ll_t - want["loglik"]) / abs(want["loglik"]),
                                                 np.abs(sc_t - want["score"]) / scale))

    def errs(t):
        return np.abs(np.array([t[1], t[4], t[5]]) - ref) / np.abs(ref)

    e0, e2 = errs(t0), errs(t2)
    say("q, u_alpha, u_nu relative error: unrefined %s refined %s" % (e0, e2))
    assert np.array_equal(t0[[0, 2, 3, 6, 7, 8]], t2[[0, 2, 3, 6, 7, 8]])
    assert np.all(e2 <= 1e-10)
    # (n = 2 is one block: no trailing update in FP32, nothing to refine)
    assert np.all(e2 <= np.maximum(1e-2 * e0, 1e-14))
    # the log-likelihood takes the refined q: only log det keeps FP32 rounding
    ll_terms = -0.5 * n * np.log(2 * np.pi) - 0.5 * t2[0] - 0.5 * t2[1]
    assert abs(ll2 - ll_terms) <= 1e-14 * abs(ll_terms)


def test_mixed_fit_switches_to_fp64(ctx):
    """Fisher-BT on a context in the mixed form: Fisher steps from mixed
    derivatives while the score is large, FP64 from the switch point on, so
    the stopping test is always taken on an FP64 score.  The result is a
    stationary point of the FP64 log-likelihood (||grad||_2 <= 1e-3 in a fresh
    FP64 evaluation) and agrees with the FP64 fit to 1e-5 relative in theta."""
    n = 2000
    say("mixed fit n=%d" % n)
    locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 2024)
    ctx.set_data(locs, z)
    r64 = ctx.fit()
    assert r64["converged"] and r64["precision_switch"] == -1
    assert r64["n_fp64_evals"] == r64["n_grad_calls"] + (1 if r64["used_nelder_mead"] else 0)
    ctx.set_precision(fbt.MIXED_FP32)
    try:
        rm = ctx.fit()
        _, g_after, _ = ctx.eval((1.0, 0.1, 0.5))      # fbt_fit restored the mixed form
        rnever = ctx.fit(mixed_switch=0.0)
    finally:
        ctx.set_precision(fbt.FP64)
    assert not np.array_equal(g_after[1:], ctx.eval((1.0, 0.1, 0.5))[1][1:])
    say("fp64", r64["theta"], r64["n_grad_calls"], "mixed", rm["theta"], rm["n_grad_calls"],
        "switch at", rm["precision_switch"], "fp64 evals", rm["n_fp64_evals"],
        "never-switch", rnever["theta"], rnever["converged"])
    assert rm["converged"] and not rm["used_nelder_mead"]
    assert 0 <= rm["precision_switch"] < rm["n_grad_calls"]
    assert rm["n_fp64_evals"] == rm["n_grad_calls"] - rm["precision_switch"]
    assert rnever["precision_switch"] == -1 and rnever["n_fp64_evals"] == 0
    ll, g, _ = ctx.eval(tuple(rm["theta"]))
    assert np.linalg.norm(g) <= 1e-3 and ll == rm["loglik"]
    np.testing.assert_allclose(rm["theta"], r64["theta"], rtol=1e-5)
