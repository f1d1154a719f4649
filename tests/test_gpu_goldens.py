"""GPU evaluations at the full sizes against stored oracle evaluations
(written by tests/golden/make_eval_goldens.py, which calls only the oracle):

  * the 20,000-point benchmark field at theta = (1, 0.1, 0.5) and at the
    oracle fit's theta-hat: log-likelihood, score, Fisher information and the
    nine intermediate terms of Algorithm 3, for both forms of the W phase
    (two-sided reduction and block solves), in the launch configuration the
    benchmark times;
  * the 10,000-point differentiation field at 20 random parameter vectors:
    the score of the adjoint form (fbt_grad) and of Algorithm 3 (fbt_eval).

Criteria (FP64): |d l| <= 1e-10 |l|; score per term |d l_i| <= 1e-10 s_i with
s_i = (|tr(Sigma^-1 Sigma_i)| + |w' Sigma_i w|) / 2 (sigma2: (q + n) / (2 sigma2)),
the size of the two terms whose difference the score is; Fisher
|d I_ij| <= 1e-8 sqrt(I_ii I_jj).  The relative score error |d l_i| / |l_i| is
printed beside it.  The 10,000-point gates apply where eps * cond_1(Sigma)
<= 1e-6 (the oracle's LAPACK condition estimate, stored with the point);
elsewhere the achieved agreement is printed.
"""
import json
import os
import sys

import numpy as np
import pytest

import paper_2601_11437_amd as fbt
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip("%s not written (tests/golden/make_eval_goldens.py)" % name)
    with open(path) as f:
        return json.load(f)


def _scales(p, n):
    th = p["theta"]
    return np.array([(p["quad"] + n) / (2 * th[0]),
                     0.5 * (abs(p["trace"]["a"]) + abs(p["wSw"]["a"])),
                     0.5 * (abs(p["trace"]["n"]) + abs(p["wSw"]["n"]))])


def _check(p, n, ll, score, fisher, terms=None, what=""):
    scale = _scales(p, n)
    want_s = np.array(p["score"])
    I = np.array(p["fisher"])
    d = np.sqrt(np.outer(np.diag(I), np.diag(I)))
    e_ll = abs(ll - p["loglik"]) / abs(p["loglik"])
    e_s = np.abs(score - want_s) / scale
    e_f = np.max(np.abs(fisher - I) / d)
    rel = np.abs(score - want_s) / np.maximum(np.abs(want_s), 1e-300)
    say("%s theta=%s  loglik %.1e  score/scale %s  score rel %s  fisher %.1e"
        % (what, np.round(p["theta"], 6).tolist(), e_ll, np.array2string(e_s, precision=1),
           np.array2string(rel, precision=1), e_f))
    assert e_ll <= 1e-10
    assert np.all(e_s <= 1e-10), e_s
    assert e_f <= 1e-8
    if terms is not None:
        ref = [p["logdet"], p["quad"], p["trace"]["a"], p["trace"]["n"], p["wSw"]["a"],
               p["wSw"]["n"], p["trAB_direct"]["aa"], p["trAB_direct"]["an"],
               p["trAB_direct"]["nn"]]
        sc = [abs(p["logdet"]) + n, p["quad"], scale[1], scale[2], scale[1], scale[2],
              2 * I[1, 1], 2 * d[1, 2], 2 * I[2, 2]]
        for k in range(9):
            assert abs(terms[k] - ref[k]) <= 1e-10 * sc[k], (k, terms[k], ref[k])


@pytest.fixture(scope="module")
def field20k():
    g = _load("eval_n20k_oracle.json")
    w = g["workload"]
    say("goldens: generating n=%d" % w["n"])
    locs, z, info = synth.dataset(w["n"], w["theta_true"], w["seed"])
    assert info["redraws"] == w["redraws"]
    ctx = fbt.Context(0)
    ctx.set_data(locs, z)
    yield ctx, g
    ctx.close()


@pytest.mark.parametrize("wphase", [fbt.WPHASE_TWO_SIDED, fbt.WPHASE_SOLVES],
                         ids=["two_sided", "solves"])
def test_eval_n20k_against_oracle(field20k, wphase):
    ctx, g = field20k
    n = g["workload"]["n"]
    ctx.set_wphase(wphase)
    try:
        for p in g["points"]:
            th = p["theta"]
            ll, score, fisher = ctx.eval(th)
            terms = ctx.eval_terms(th)
            _check(p, n, ll, score, fisher, terms, "n20k wphase=%d" % wphase)
    finally:
        ctx.set_wphase(fbt.WPHASE_TWO_SIDED)


def test_score_n10k_against_oracle():
    g = _load("eval_n10k_oracle.json")
    w = g["workload"]
    n = w["n"]
    say("goldens: generating n=%d" % n)
    locs, z, info = synth.dataset(n, w["theta_true"], w["seed"])
    assert info["redraws"] == w["redraws"]
    gated = 0
    with fbt.Context(0) as ctx:
        ctx.set_data(locs, z)
        for p in g["points"]:
            th = p["theta"]
            gate = np.finfo(float).eps * p["cond1"] <= 1e-6
            scale = _scales(p, n)
            want_s = np.array(p["score"])
            lla, sa = ctx.grad(th)
            ll, sw, fisher = ctx.eval(th)
            e_adj = np.max(np.abs(sa - want_s) / scale)
            e_w = np.max(np.abs(sw - want_s) / scale)
            e_ll = max(abs(lla - p["loglik"]), abs(ll - p["loglik"])) / abs(p["loglik"])
            I = np.array(p["fisher"])
            d = np.sqrt(np.outer(np.diag(I), np.diag(I)))
            e_f = np.max(np.abs(fisher - I) / d)
            say("n10k theta=%s cond1=%.1e  loglik %.1e  adjoint %.1e  W-route %.1e  fisher %.1e  %s"
                % (np.round(th, 4).tolist(), p["cond1"], e_ll, e_adj, e_w, e_f,
                   "gated" if gate else "reported only"))
            if gate:
                gated += 1
                assert e_ll <= 1e-10
                assert e_adj <= 1e-10
                assert e_w <= 1e-10
                assert e_f <= 1e-8
    say("n10k: %d of %d points gated" % (gated, len(g["points"])))
    assert gated >= 1
