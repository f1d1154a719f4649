"""The allocation-free entry point fbt_eval_noalloc (through the C ABI)
against fbt_eval on a context, on the same seeded inputs: two calls in a row,
the second with a smaller field, each equal to the context's result to the
FP64 parity bar (log-likelihood 1e-10 relative, score 1e-10 of its per-term
scale, Fisher 1e-8 of sqrt(I_ii I_jj)); the launch sequence is fbt_eval's on
one stream, so equality is expected bitwise and checked as well.  Argument
errors are rejected before any launch; a non-finite observation is caught by
the packing kernel's own check."""
import ctypes
import sys

import numpy as np
import pytest

import paper_2601_11437_amd as fbt
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(locs, z, theta, stream=None):
    import torch

    dl = torch.tensor(np.ascontiguousarray(locs), dtype=torch.float64, device="cuda")
    dz = torch.tensor(np.ascontiguousarray(z), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ll = ctypes.c_double()
    score = np.zeros(3)
    fisher = np.zeros(9)
    st = fbt.lib().fbt_eval_noalloc(0, stream, len(z), dl.data_ptr(), dz.data_ptr(),
                                    th.ctypes.data, ctypes.addressof(ll), score.ctypes.data,
                                    fisher.ctypes.data)
    return st, ll.value, score, fisher.reshape(3, 3)


def _context_eval(locs, z, theta, terms=False):
    with fbt.Context(0) as ctx:
        ctx.set_data(locs, z)
        r = ctx.eval(theta)
        return (r, ctx.eval_terms(theta)) if terms else r


@pytest.mark.parametrize("sizes", [(1000, 300), (1023, 1)])
def test_noalloc_matches_eval(sizes):
    import torch

    stream = torch.cuda.current_stream().cuda_stream
    for k, n in enumerate(sizes):
        theta = (1.2, 0.08, 0.9) if k == 0 else (0.7, 0.12, 1.6)
        say("noalloc n=%d theta=%s" % (n, theta))
        locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 7000 + n)
        st, ll, score, fisher = _noalloc(locs, z, theta, stream)
        assert st == fbt.OK, st
        (rll, rscore, rfisher), t = _context_eval(locs, z, theta, terms=True)
        assert abs(ll - rll) <= 1e-10 * abs(rll)
        scale = np.array([(t[1] + n) / (2 * theta[0]), 0.5 * (abs(t[2]) + abs(t[4])),
                          0.5 * (abs(t[3]) + abs(t[5]))])
        assert np.all(np.abs(score - rscore) <= 1e-10 * scale), (score, rscore)
        d = np.sqrt(np.outer(np.diag(rfisher), np.diag(rfisher)))
        assert np.all(np.abs(fisher - rfisher) <= 1e-8 * d)
        assert ll == rll and np.array_equal(score, rscore) and np.array_equal(fisher, rfisher)


def test_noalloc_rejects_bad_arguments():
    locs, z, _ = synth.dataset(50, (1.0, 0.1, 0.5), 77)
    theta = (1.0, 0.1, 0.5)
    assert _noalloc(locs, z, (1.0, -0.1, 0.5))[0] == fbt.EINVAL
    big_locs = np.zeros((fbt_max() + 1, 2))
    big_z = np.zeros(fbt_max() + 1)
    assert _noalloc(big_locs, big_z, theta)[0] == fbt.EINVAL
    bad = z.copy()
    bad[7] = np.nan
    assert _noalloc(locs, bad, theta)[0] == fbt.EINVAL
    # the scratch is usable again after a rejected call
    st, ll, _, _ = _noalloc(locs, z, theta)
    assert st == fbt.OK
    assert ll == _context_eval(locs, z, theta)[0]


def fbt_max():
    return 1023
