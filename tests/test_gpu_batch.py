"""Batched fields (fbt_batch_*) through the C ABI: each field's result must be
bitwise the single-context result for that field, whatever the number of
workers; a field whose covariance is not positive definite reports
FBT_ENOTPD in its status slot without disturbing the others; skipped fields
are untouched.  Field sizes are drawn so that several fall in different
padded orders (npad = 256 ceil((n + 1) / 256)) and buffers are reused across
sizes."""
import json
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


@pytest.mark.parametrize("precision", [fbt.MIXED_FP32, fbt.MIXED_BF16, fbt.MIXED_FP32_ALL,
                                       fbt.MIXED_BF16_ALL])
def test_batch_mixed_matches_single_context(fields, precision):
    """The mixed forms in batched groups (per-field strides of the FP32 operand
    copies, for the FP32 forms) give bitwise the single-context results; in
    the low-precision Cholesky forms a field whose factorisation fails has the
    same status in both."""
    data, thetas = fields
    nf = len(data)
    mode = np.array([2, 1] * nf)[:nf]
    mode[3] = 0                       # the non-PD field is covered by the FP64 test
    ref_ll, ref_sc, ref_fi = np.full(nf, np.nan), np.full((nf, 3), np.nan), np.full((nf, 3, 3), np.nan)
    ref_st = np.zeros(nf, dtype=np.int32)
    with fbt.Context(0) as c:
        c.set_precision(precision)
        for f, (locs, z) in enumerate(data):
            if mode[f] == 0:
                continue
            c.set_data(locs, z)
            try:
                if mode[f] == 1:
                    ref_ll[f] = c.loglik(thetas[f])
                else:
                    ref_ll[f], ref_sc[f], ref_fi[f] = c.eval(thetas[f])
            except fbt.FisherBTError as e:
                ref_st[f] = e.status
    say("batch precision=%d, %d fields fail to factor" % (precision, np.count_nonzero(ref_st)))
    if precision in (fbt.MIXED_FP32, fbt.MIXED_BF16):
        assert np.all(ref_st == 0)
    b = fbt.Batch(3, precision=precision)
    b.set_fields(data)
    ll, sc, fi, st = b.eval(thetas, mode)
    b.close()
    np.testing.assert_array_equal(st, ref_st)
    np.testing.assert_array_equal(ll, ref_ll)
    np.testing.assert_array_equal(sc, ref_sc)
    np.testing.assert_array_equal(fi, ref_fi)


def _calls(thetas0, nf):
    g = synth.rng(77)
    calls = [thetas0]
    for _ in range(2):
        th = thetas0.copy()
        th[:, 0] *= g.uniform(0.8, 1.2, nf)
        th[:, 1] *= g.uniform(0.8, 1.2, nf)
        th[3] = thetas0[3]
        calls.append(th)
    return calls


@pytest.mark.skip(reason="the graph execution is switched off: its first capture and replay "
                         "crashed the host process (segmentation fault) and the cause is not "
                         "identified")
def test_graph_execution_matches_workers(fields):
    """The whole call captured in one HIP graph and replayed: every replay
    (three calls with different theta, eager work of another batch and a
    single-context evaluation between them, a non-PD field, skipped and
    adjoint-mode fields) is bitwise the worker execution's result."""
    data, thetas0 = fields
    nf = len(data)
    mode = np.array([2, 1, 3] * (nf // 3 + 1))[:nf]
    mode[5] = 0
    g = synth.rng(77)
    calls = [thetas0]
    for _ in range(2):
        th = thetas0.copy()
        th[:, 0] *= g.uniform(0.8, 1.2, nf)
        th[:, 1] *= g.uniform(0.8, 1.2, nf)
        th[3] = thetas0[3]
        calls.append(th)
    bw, bg = fbt.Batch(3), fbt.Batch(2)
    bw.set_fields(data)
    bg.set_fields(data)
    bg.set_exec(fbt.Batch.GRAPH)
    assert bg.exec == fbt.Batch.GRAPH
    for r, th in enumerate(calls * 2):
        say("graph replay %d" % r)
        want = bw.eval(th, mode)
        got = bg.eval(th, mode)
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)
        assert got[3][3] == fbt.ENOTPD and np.isnan(got[0][5])
        with fbt.Context(0) as c:       # eager work between replays
            c.set_data(*data[0])
            c.loglik(th[0])
    bw.close()
    bg.close()


def test_graph_execution_is_refused(fields):
    data, _ = fields
    b = fbt.Batch(1)
    b.set_fields(data[:2])
    with pytest.raises(fbt.FisherBTError):
        b.set_exec(fbt.Batch.GRAPH)
    assert b.exec == fbt.Batch.WORKERS
    b.close()


def test_group_limits_and_autotune(fields, tmp_path):
    """Group limits change the grouping, not the numbers (bitwise); the
    autotuner picks a limit per padded order and its file restores them."""
    data, thetas0 = fields
    nf = len(data)
    mode = np.array([2, 1, 3] * (nf // 3 + 1))[:nf]
    mode[5] = 0
    calls = _calls(thetas0, nf)
    bw, bl = fbt.Batch(3), fbt.Batch(2)
    bw.set_fields(data)
    bl.set_fields(data)
    # limits: one field per group of order 768, two for 1280
    bl.set_group_limit(768, 1)
    bl.set_group_limit(1280, 2)
    assert bl.group_limit(768) == 1 and bl.group_limit(512) == 0
    for th in calls:
        got = bl.eval(th, mode)
        want = bw.eval(th, mode)
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)
    # autotuner on a small workload, its file restores the choices
    path = tmp_path / "tune.json"
    small = [i for i in range(nf) if data[i][1].size <= 700]
    bt = fbt.Batch(2)
    bt.set_fields([data[i] for i in small])
    bt.autotune(calls[0][small], 2, path)
    rec = json.loads(path.read_text())
    say("autotune", rec)
    assert rec["exec"] in (0, 2) and rec["chosen"] in ("per_order", "none", "all_4", "all_16",
                                                       "all_64")
    assert rec["seconds_persistent_64"] > 0 and rec["seconds_persistent_128"] > 0
    if rec["exec"] == 2:
        assert rec["tile"] in (64, 128)
    # "none" stores no limit, "all_N" stores N for every order; "per_order"
    # may store none either, when no limit was fastest for every order
    if rec["chosen"] == "none":
        assert len(rec["limits"]) == 0
    elif rec["chosen"] != "per_order":
        want_u = int(rec["chosen"][4:])
        assert rec["limits"] and all(v == want_u for v in rec["limits"].values())
    bt2 = fbt.Batch(2)
    bt2.set_fields([data[i] for i in small])
    bt2.load_tuning(path)
    assert bt2.exec == rec["exec"]
    if rec["exec"] == 2:
        assert bt2.tile == rec["tile"]
    for k, v in rec["limits"].items():
        assert bt2.group_limit(int(k)) == v
    a = bt2.eval(calls[0][small], 2)
    mode_s = np.zeros(nf, dtype=np.int32)
    mode_s[small] = 2
    b = bw.eval(calls[0], mode_s)
    if rec["exec"] == 0:
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y[small])
    else:
        # the persistent execution: the same statuses, log-likelihoods to
        # rounding (its blocking differs)
        np.testing.assert_array_equal(a[3], b[3][small])
        ok = a[3] == fbt.OK
        np.testing.assert_allclose(a[0][ok], b[0][small][ok], rtol=1e-9)
    for bb in (bw, bl, bt, bt2):
        bb.close()


def test_batch_argument_errors(fields):
    data, thetas = fields
    b = fbt.Batch(2)
    b.set_fields(data[:3])
    with pytest.raises(fbt.FisherBTError):
        b.eval(thetas[:3], [2, 2, 7])
    b.close()


def test_batch_fields_against_oracle(oracle_mod):
    """Four fields of the many-field workload (n_f ~ U[500, 4000], theta_f
    drawn as there) evaluated in one batched call, each against the oracle at
    the FP64 parity bar: loglik 1e-10 relative, score 1e-10 of its per-term
    scale, Fisher 1e-8 of sqrt(I_ii I_jj).  The four are the workload's first
    fields with n below 1,500 (the oracle's cost) whose covariance at theta_f
    has eps cond(Sigma) <= 1e-8: the workload's draws reach cond ~ 1e15, and
    at cond = 1.5e9 (eps cond = 3e-7) the loglik already differs by 1.2e-10
    relative (measured; rounding amplified by the conditioning)."""
    g = synth.rng(5000)
    ns = g.integers(500, 4001, 256)
    thetas_all = synth.batch_redraw_thetas(np.zeros((256, 3)), np.ones(256, bool), g)
    data, thetas, pick = [], [], []
    for f in range(256):
        if ns[f] >= 1500:
            continue
        locs, z, _ = synth.dataset(int(ns[f]), (1.0, 0.1, 0.5), 5001 + f)
        kappa = np.linalg.cond(oracle_mod.cov_matrices(locs, thetas_all[f], which=("S",))[0])
        say("field %d n=%d theta=%s cond=%.1e" % (f, ns[f], np.round(thetas_all[f], 4), kappa))
        if np.finfo(float).eps * kappa > 1e-8:
            continue
        data.append((locs, z))
        thetas.append(thetas_all[f])
        pick.append(f)
        if len(pick) == 4:
            break
    thetas = np.array(thetas)
    say("batch vs oracle: fields %s, n %s" % (pick, [int(ns[f]) for f in pick]))
    b = fbt.Batch(2)
    b.set_fields(data)
    ll, sc, fi, st = b.eval(thetas, fbt.Batch.EVAL)
    b.close()
    assert len(pick) == 4
    for k, (locs, z) in enumerate(data):
        th = thetas[k]
        want = oracle_mod.evaluate(locs, z, th)
        n = z.size
        assert st[k] == fbt.OK
        scale = np.array([(want["quad"] + n) / (2 * th[0]),
                          0.5 * (abs(want["trace"]["a"]) + abs(want["wSw"]["a"])),
                          0.5 * (abs(want["trace"]["n"]) + abs(want["wSw"]["n"]))])
        I = want["fisher"]
        d = np.sqrt(np.outer(np.diag(I), np.diag(I)))
        say("field %d: loglik %.1e score/scale %s fisher %.1e"
            % (pick[k], abs(ll[k] - want["loglik"]) / abs(want["loglik"]),
               np.array2string(np.abs(sc[k] - want["score"]) / scale, precision=1),
               np.max(np.abs(fi[k] - I) / d)))
        assert abs(ll[k] - want["loglik"]) <= 1e-10 * abs(want["loglik"])
        assert np.all(np.abs(sc[k] - want["score"]) <= 1e-10 * scale)
        assert np.all(np.abs(fi[k] - I) <= 1e-8 * d)
