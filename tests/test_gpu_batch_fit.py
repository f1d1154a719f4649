"""Batched Fisher-BT (fbt_batch_fit): Algorithm 1 for many fields at once,
one evaluation round (one persistent launch) per iteration of the fits.
Each field's fit must take the oracle's path - the same numbers of
log-likelihood and derivative evaluations - and reach the oracle's theta-hat
to 1e-6 relative where the oracle's fit converges by scoring (the driver is
the same Algorithm 1; the evaluations agree to ~1e-12), and agree with the
single-field GPU fit."""
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
def fields():
    return synth.batch_fit_workload(nf=6, seed=9300, n_range=(300, 500))


def test_batch_fit_against_oracle(fields, oracle_mod):
    data, theta_true = fields
    b = fbt.Batch(1)
    b.set_fields(data)
    b.set_exec(fbt.Batch.PERSISTENT)
    say("batched fit of %d fields, n %s" % (len(data), [z.size for _, z in data]))
    fits, st, rounds = b.fit()
    b.close()
    say("  rounds %d" % rounds)
    assert rounds > 0
    converged = 0
    for f, (locs, z) in enumerate(data):
        want = oracle_mod.fisher_bt(oracle_mod.OracleEvaluator(locs, z))
        got = fits[f]
        rel = np.abs(got["theta"] - want["theta"]) / np.abs(want["theta"])
        say("  field %d n=%d: theta %s oracle %s rel %.1e calls %d/%d oracle %d/%d nm %s/%s"
            % (f, z.size, np.round(got["theta"], 6), np.round(want["theta"], 6), rel.max(),
               got["n_loglik_calls"], got["n_grad_calls"], want["n_loglik_calls"],
               want["n_grad_calls"], got["used_nelder_mead"], want["used_nelder_mead"]))
        assert st[f] == fbt.OK
        if want["converged"] and not want["used_nelder_mead"]:
            converged += 1
            assert got["converged"] and not got["used_nelder_mead"]
            assert got["n_loglik_calls"] == want["n_loglik_calls"]
            assert got["n_grad_calls"] == want["n_grad_calls"]
            assert rel.max() <= 1e-6
        # every round serves each unfinished fit one evaluation
        assert rounds >= got["n_grad_calls"]
    assert converged >= 4


def test_batch_fit_matches_single_field_fits(fields):
    """The batched fit of a subset (active mask, given starts) against
    fbt_fit on a context, field by field: the same path and theta-hat to
    1e-8 (two FP64 evaluations of the same field, different blockings)."""
    data, theta_true = fields
    nf = len(data)
    active = np.array([1, 0, 1, 1, 0, 1], dtype=bool)
    t0 = np.array(theta_true) * 1.3
    b = fbt.Batch(1)
    b.set_fields(data)
    b.set_exec(fbt.Batch.PERSISTENT)
    say("batched fit with starts, fields %s" % np.flatnonzero(active).tolist())
    fits, st, rounds = b.fit(theta0=t0, active=active)
    b.close()
    for f in range(nf):
        if not active[f]:
            assert fits[f] is None
            continue
        with fbt.Context(0) as c:
            c.set_data(*data[f])
            ref = c.fit(theta0=t0[f])
        got = fits[f]
        rel = np.abs(got["theta"] - ref["theta"]) / np.abs(ref["theta"])
        say("  field %d: rel %.1e calls %d/%d single %d/%d"
            % (f, rel.max(), got["n_loglik_calls"], got["n_grad_calls"], ref["n_loglik_calls"],
               ref["n_grad_calls"]))
        assert got["status"] == ref["status"]
        assert (got["n_loglik_calls"], got["n_grad_calls"]) == (ref["n_loglik_calls"],
                                                               ref["n_grad_calls"])
        assert rel.max() <= 1e-8


def test_batch_fit_with_few_threads(fields):
    """Two fits at a time (the others start as those end): every field's
    result bitwise the one of the run with all fits at once."""
    data, theta_true = fields
    out = []
    for threads in (0, 2):
        b = fbt.Batch(1)
        b.set_fields(data)
        b.set_exec(fbt.Batch.PERSISTENT)
        b.set_fit_threads(threads)
        say("batched fit, %d fits at once" % (threads or len(data)))
        out.append(b.fit())
        b.close()
    (a, sa, ra), (c, sc, rc) = out
    say("  rounds %d and %d" % (ra, rc))
    assert rc > ra
    np.testing.assert_array_equal(sa, sc)
    for x, y in zip(a, c):
        for k in ("theta", "loglik", "score", "fisher", "n_loglik_calls", "n_grad_calls"):
            np.testing.assert_array_equal(x[k], y[k])


@pytest.mark.parametrize("precision", [fbt.MIXED_FP32_ALL, fbt.MIXED_BF16_ALL])
def test_batch_fit_refuses_low_precision_cholesky(fields, precision):
    """As fbt_fit, the batched fit refuses the forms whose log-likelihood
    carries low-precision Cholesky rounding (FBT_EINVAL, with the reason)."""
    data, _ = fields
    b = fbt.Batch(1, precision=precision)
    b.set_fields(data[:2])
    with pytest.raises(fbt.FisherBTError) as e:
        b.fit()
    assert e.value.status == fbt.EINVAL and "Cholesky" in str(e.value)
    b.close()
