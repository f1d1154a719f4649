"""The persistent execution of batched fields (FBT_BATCH_PERSISTENT: every
field of a call in one launch of the tile-task kernel) through the C ABI,
against the oracle at the FP64 parity bar (loglik 1e-10 relative, score
1e-10 of its per-term scale, Fisher 1e-8 of sqrt(I_ii I_jj)), for both tile
sizes and for sizes around the tile edges (n + 1 = 64, 65, 128, 129: the
observation row opens a new tile), and against the worker execution on the
many-field workload."""
import sys

import numpy as np
import pytest

import paper_2601_11437_amd as fbt
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check(k, got, want, th, n):
    ll, sc, fi = got
    assert abs(ll - want["loglik"]) <= 1e-10 * abs(want["loglik"]), (k, ll, want["loglik"])
    if sc is None:
        return
    scale = np.array([(want["quad"] + n) / (2 * th[0]),
                      0.5 * (abs(want["trace"]["a"]) + abs(want["wSw"]["a"])),
                      0.5 * (abs(want["trace"]["n"]) + abs(want["wSw"]["n"]))])
    I = want["fisher"]
    d = np.sqrt(np.outer(np.diag(I), np.diag(I)))
    with np.errstate(invalid="ignore", divide="ignore"):
        say("  field %d n=%d: loglik %.1e score/scale %s fisher %.1e"
            % (k, n, abs(ll - want["loglik"]) / abs(want["loglik"]),
               np.array2string(np.abs(sc - want["score"]) / scale, precision=1),
               np.nanmax(np.where(d > 0, np.abs(fi - I) / np.where(d > 0, d, 1), 0))))
    assert np.all(np.abs(sc - want["score"]) <= 1e-10 * scale), (k, sc, want["score"])
    assert np.all(np.abs(fi - I) <= 1e-8 * d), (k, fi, I)


@pytest.fixture(scope="module")
def small_fields():
    ns = [1, 5, 62, 63, 64, 127, 128, 129, 300, 700]
    g = synth.rng(7100)
    data, thetas = [], []
    for f, n in enumerate(ns):
        locs, z, _ = synth.dataset(n, (1.0, 0.1, 0.5), 7200 + f)
        data.append((locs, z))
        thetas.append((g.uniform(0.5, 2.0), g.uniform(0.03, 0.12), g.uniform(0.3, 1.4)))
    return data, np.array(thetas)


@pytest.mark.parametrize("tile", [64, 128])
def test_round_against_oracle(small_fields, tile, oracle_mod):
    data, thetas = small_fields
    nf = len(data)
    mode = np.array([2, 1] * nf)[:nf]
    mode[-1] = 2
    say("persistent round, tile %d, n %s" % (tile, [z.size for _, z in data]))
    b = fbt.Batch(1)
    b.set_fields(data)
    b.set_exec(fbt.Batch.PERSISTENT)
    b.set_tile(tile)
    ll, sc, fi, st = b.eval(thetas, mode)
    ntasks, est, ms = b.round_stats()
    say("  tasks %d, kernel %.3f ms" % (ntasks, ms))
    b.close()
    assert ntasks > 0 and ms > 0
    for k, (locs, z) in enumerate(data):
        assert st[k] == fbt.OK, (k, st[k])
        th = thetas[k]
        if mode[k] == 1:
            want = {"loglik": oracle_mod.loglik(locs, z, th)["loglik"]}
            _check(k, (ll[k], None, None), want, th, z.size)
        else:
            want = oracle_mod.evaluate(locs, z, th)
            _check(k, (ll[k], sc[k], fi[k]), want, th, z.size)


def test_round_status_and_repeat(small_fields, oracle_mod):
    """A skipped field, an invalid theta (FBT_EINVAL in its slot), a
    numerically indefinite covariance (FBT_ENOTPD) and an adjoint-mode field
    (run after the launch) beside ordinary ones; then a second call with other
    theta on the same plan, and a third with other modes (a new plan)."""
    data, thetas = small_fields
    locs_bad, z_bad, _ = synth.dataset(400, (1.0, 0.1, 0.5), 7300)
    data2 = list(data[6:]) + [(locs_bad, z_bad)]
    th = np.array(list(thetas[6:]) + [(1.0, 50.0, 4.0)])
    nf = len(data2)
    mode = np.array([2, 0, 1, 3, 2])
    th[0] = (-1.0, 0.1, 0.5)
    b = fbt.Batch(1)
    b.set_fields(data2)
    b.set_exec(fbt.Batch.PERSISTENT)
    say("persistent round: status cases")
    ll, sc, fi, st = b.eval(th, mode)
    assert st.tolist() == [fbt.EINVAL, fbt.OK, fbt.OK, fbt.OK, fbt.ENOTPD], st
    assert np.isnan(ll[1]) and np.isnan(ll[0]) and np.isnan(ll[4])
    _check(2, (ll[2], None, None), {"loglik": oracle_mod.loglik(*data2[2], th[2])["loglik"]}, th[2],
           data2[2][1].size)
    with fbt.Context(0) as c:
        c.set_data(*data2[3])
        ref = c.grad(th[3])
    assert ll[3] == ref[0] and np.array_equal(sc[3], ref[1])
    for rep, md in enumerate(([2, 2, 2, 1, 0], [1, 2, 0, 2, 0])):
        th2 = np.array(thetas[6:10].tolist() + [(1.0, 0.1, 0.5)]) * (1.0 + 0.05 * (rep + 1))
        say("persistent round: call %d, modes %s" % (rep + 2, md))
        ll, sc, fi, st = b.eval(th2, md)
        for k in range(nf):
            if md[k] == 0:
                assert np.isnan(ll[k])
                continue
            assert st[k] == fbt.OK, (k, st[k])
            locs, z = data2[k]
            if md[k] == 1:
                _check(k, (ll[k], None, None), {"loglik": oracle_mod.loglik(locs, z, th2[k])["loglik"]},
                       th2[k], z.size)
            else:
                _check(k, (ll[k], sc[k], fi[k]), oracle_mod.evaluate(locs, z, th2[k]), th2[k],
                       z.size)
    b.close()


def test_round_fields_against_oracle(oracle_mod):
    """The four fields of the many-field workload that the worker execution's
    oracle test uses (n below 1,500, eps cond(Sigma) <= 1e-8), in one
    persistent call with both tile sizes."""
    g = synth.rng(5000)
    ns = g.integers(500, 4001, 256)
    thetas_all = synth.batch_redraw_thetas(np.zeros((256, 3)), np.ones(256, bool), g)
    data, thetas, pick = [], [], []
    for f in range(256):
        if ns[f] >= 1500:
            continue
        locs, z, _ = synth.dataset(int(ns[f]), (1.0, 0.1, 0.5), 5001 + f)
        kappa = np.linalg.cond(oracle_mod.cov_matrices(locs, thetas_all[f], which=("S",))[0])
        if np.finfo(float).eps * kappa > 1e-8:
            continue
        data.append((locs, z))
        thetas.append(thetas_all[f])
        pick.append(f)
        if len(pick) == 4:
            break
    thetas = np.array(thetas)
    wants = [oracle_mod.evaluate(locs, z, th) for (locs, z), th in zip(data, thetas)]
    for tile in (64, 128):
        say("persistent round vs oracle: fields %s, tile %d" % (pick, tile))
        b = fbt.Batch(1)
        b.set_fields(data)
        b.set_exec(fbt.Batch.PERSISTENT)
        b.set_tile(tile)
        ll, sc, fi, st = b.eval(thetas, fbt.Batch.EVAL)
        b.close()
        for k, (locs, z) in enumerate(data):
            assert st[k] == fbt.OK
            _check(pick[k], (ll[k], sc[k], fi[k]), wants[k], thetas[k], z.size)


def test_round_many_field_workload():
    """256 fields, n ~ U[500, 4000], theta drawn as in the batched workload:
    one persistent call per tile size against the worker execution.  Both are
    FP64 with different blockings, so they agree to the conditioning of each
    field: statuses must be equal, and log-likelihoods agree to 1e-10
    relative for every field whose two results agree on the score to 1e-6 of
    its scale (the well-conditioned ones; the count is printed)."""
    g = synth.rng(5000)
    ns = g.integers(500, 4001, 256)
    thetas = synth.batch_redraw_thetas(np.zeros((256, 3)), np.ones(256, bool), g)
    data = [synth.dataset(int(ns[f]), (1.0, 0.1, 0.5), 5001 + f)[:2] for f in range(256)]
    say("many-field workload: worker execution")
    b = fbt.Batch(2)
    b.set_fields(data)
    ref = b.eval(thetas, fbt.Batch.EVAL)
    b.set_exec(fbt.Batch.PERSISTENT)
    for tile in (64, 128):
        say("many-field workload: persistent, tile %d" % tile)
        b.set_tile(tile)
        ll, sc, fi, st = b.eval(thetas, fbt.Batch.EVAL)
        ntasks, est, ms = b.round_stats()
        say("  tasks %d, planner %.1f ms, kernel %.1f ms" % (ntasks, est / 1e3, ms))
        np.testing.assert_array_equal(st, ref[3])
        ok = st == fbt.OK
        rel = np.abs(ll[ok] - ref[0][ok]) / np.abs(ref[0][ok])
        say("  loglik relative difference: median %.1e, max %.1e" % (np.median(rel), rel.max()))
        assert np.median(rel) <= 1e-10
    b.close()


def test_round_graph_replays(small_fields):
    """The persistent round replayed from a HIP graph: every replay, with other
    eager work and synchronisations between the replays, gives bitwise the
    direct launch's results for the same theta."""
    data, thetas = small_fields
    nf = len(data)
    mode = np.array([2, 1] * nf)[:nf]
    calls = [thetas * (1.0 + 0.03 * k) for k in range(3)]
    direct = fbt.Batch(1)
    direct.set_fields(data)
    direct.set_exec(fbt.Batch.PERSISTENT)
    direct.set_round_graph(False)
    want = [direct.eval(th, mode) for th in calls]
    g = fbt.Batch(1)
    g.set_fields(data)
    g.set_exec(fbt.Batch.PERSISTENT)
    g.set_round_graph(True)
    for rep in range(2):
        for k, th in enumerate(calls):
            say("graph replay %d, theta set %d" % (rep, k))
            got = g.eval(th, mode)
            direct.eval(calls[(k + 1) % 3], mode)   # eager work between replays
            for a, b in zip(got, want[k]):
                np.testing.assert_array_equal(a, b)
    g.close()
    direct.close()
