"""The Nelder-Mead branch of Algorithm 1 on the GPU against the oracle's
driver on the oracle's evaluations.  The scoring budget is cut so that the
fit shifts to Nelder-Mead (the paper's shift rule): up to the shift both take
the same path (the same calls, the same point), and Nelder-Mead then reaches
the same optimum.  Its simplex branches on comparisons of log-likelihoods
that the two sides agree on only to rounding, so the optimum is compared
(log-likelihood 1e-9 relative, theta 1e-4), not the path after the shift.
Both the single-field fit and the batched fit (one persistent launch per
round) are checked."""
import sys

import numpy as np
import pytest

import paper_2601_11437_amd as fbt
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [(400, (1.0, 0.1, 0.5), 11, 3), (350, (1.5, 0.05, 1.2), 12, 2)]


@pytest.mark.parametrize("n,theta_true,seed,max_grad", CASES)
def test_nelder_mead_branch_against_oracle(n, theta_true, seed, max_grad, oracle_mod):
    locs, z, _ = synth.dataset(n, theta_true, seed)
    want = oracle_mod.fisher_bt(oracle_mod.OracleEvaluator(locs, z), max_grad_calls=max_grad)
    assert want["used_nelder_mead"], "the cut budget must force the shift"
    say("n=%d: oracle theta %s ll %.12f (%d ll, %d grad)"
        % (n, np.round(want["theta"], 8), want["loglik"], want["n_loglik_calls"],
           want["n_grad_calls"]))
    with fbt.Context(0) as c:
        c.set_data(locs, z)
        got = c.fit(max_grad_calls=max_grad)
    b = fbt.Batch(1)
    b.set_fields([(locs, z)])
    b.set_exec(fbt.Batch.PERSISTENT)
    fits, st, rounds = b.fit(max_grad_calls=max_grad)
    b.close()
    for name, r in (("single", got), ("batched", fits[0])):
        say("  %s: theta %s ll %.12f (%d ll, %d grad, %d NM evals)"
            % (name, np.round(r["theta"], 8), r["loglik"], r["n_loglik_calls"],
               r["n_grad_calls"], r["n_nm_evals"]))
        assert r["used_nelder_mead"]
        # the scoring part up to the shift: same derivative calls
        assert r["n_grad_calls"] == want["n_grad_calls"]
        assert abs(r["loglik"] - want["loglik"]) <= 1e-9 * abs(want["loglik"])
        np.testing.assert_allclose(r["theta"], want["theta"], rtol=1e-4)
