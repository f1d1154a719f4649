"""Batched fields (fbt_batch_*) through the C ABI: each field's result must be
bitwise the single-context result for that field, whatever the number of
workers; a field whose covariance is not positive definite reports
FBT_ENOTPD in its status slot without disturbing the others; skipped fields
are untouched.  Field sizes are drawn so that several fall in different
padded orders (npad = 256 ceil((n + 1) / 256)) and buffers are reused across
sizes."""
import sys

import numpy as np
import pytest

import paper_2601_11437_amd as fbt
from paper_2601_11437_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fields():
    g = synth.rng(5000)
    ns = [int(v) for v in g.integers(200, 1300, 14)] + [255, 256, 257, 1]
    out, thetas = [], []
    for f, n in enumerate(ns):
        locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 6000 + f)
        out.append((locs, z))
        thetas.append((g.uniform(0.5, 2.0), g.uniform(0.02, 0.2), g.uniform(0.3, 2.0)))
    thetas[3] = (1.0, 50.0, 4.0)      # numerically indefinite (checked in the parity tests)
    return out, np.array(thetas)


def test_batch_matches_single_context(fields):
    data, thetas = fields
    nf = len(data)
    mode = np.array([2, 1, 3] * (nf // 3 + 1))[:nf]
    mode[5] = 0
    ref_ll, ref_sc, ref_fi, ref_st = np.full(nf, np.nan), np.full((nf, 3), np.nan), \
        np.full((nf, 3, 3), np.nan), np.zeros(nf, dtype=np.int32)
    with fbt.Context(0) as c:
        for f, (locs, z) in enumerate(data):
            if mode[f] == 0:
                continue
            c.set_data(locs, z)
            try:
                if mode[f] == 1:
                    ref_ll[f] = c.loglik(thetas[f])
                elif mode[f] == 2:
                    ref_ll[f], ref_sc[f], ref_fi[f] = c.eval(thetas[f])
                else:
                    ref_ll[f], ref_sc[f] = c.grad(thetas[f])
            except fbt.FisherBTError as e:
                ref_st[f] = e.status
    assert ref_st[3] == fbt.ENOTPD
    for workers in (1, 6):
        say("batch workers=%d" % workers)
        b = fbt.Batch(workers)
        b.set_fields(data)
        ll, sc, fi, st = b.eval(thetas, mode)
        b.close()
        np.testing.assert_array_equal(st, ref_st)
        np.testing.assert_array_equal(ll, ref_ll)
        np.testing.assert_array_equal(sc, ref_sc)
        np.testing.assert_array_equal(fi, ref_fi)
        assert np.isnan(ll[5])


def test_batch_argument_errors(fields):
    data, thetas = fields
    b = fbt.Batch(2)
    b.set_fields(data[:3])
    with pytest.raises(fbt.FisherBTError):
        b.eval(thetas[:3], [2, 2, 7])
    b.close()
