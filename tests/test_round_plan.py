"""Host-only checks of the persistent execution's plan (no GPU).

The batched round runs as tile tasks in one launch; its workgroups take the
tasks in the planner's ticket order and wait on counters (the kernel's waits,
read here through fbt_round_task_deps).  Three properties are checked against
a model of the data each task reads and writes, written here from the
algorithm (left-looking tile Cholesky of the bordered covariance, forward
substitution of [Sigma_alpha | Sigma_nu], W = X L^{-T} in place of X):

* the ticket order holds every task of every field exactly once;
* in ticket order every task comes after the tasks that write what it reads,
  and after every reader of the tiles it overwrites;
* any interleaving that the counters allow (random schedules of up to 600
  workgroups, each holding one ticket at a time) runs every task only after
  those same tasks, and never deadlocks.
"""
import random

import numpy as np
import pytest

import paper_2601_11437_amd as fbt

GEN, CHOL, LSOLVE, RSOLVE, REDUCE = range(5)


def _tiles(n, bt):
    return (n + 1 + bt - 1) // bt


def expected_tasks(T, mode):
    out = set()
    if mode not in (1, 2):
        return out
    for i in range(T):
        for j in range(i + 1):
            out.add((GEN, i, j))
            out.add((CHOL, i, j))
            if mode == 2:
                out.add((RSOLVE, i, j))
    if mode == 2:
        for k in range(T):
            for c in range(2 * T):
                out.add((LSOLVE, k, c))
    out.add((REDUCE, 0, 0))
    return out


def predecessors(task, T, mode):
    """Tasks that must be finished before `task` reads its inputs or
    overwrites a tile (phase 0), and, for CHOL(i > j), before the product with
    the diagonal inverse (phase 1)."""
    ty, i, j = task
    p0, p1 = set(), set()
    if ty == CHOL:
        p0.add((GEN, i, j))
        for k in range(j):                    # L_ik, L_jk of the finished columns
            p0.add((CHOL, i, k))
            p0.add((CHOL, j, k))
        if i > j:
            p1.add((CHOL, j, j))              # L_jj^{-1}
    elif ty == LSOLVE:
        c = j % T
        p0.add((GEN, max(i, c), min(i, c)))   # the Sigma_alpha / Sigma_nu tile
        for m in range(i + 1):
            p0.add((CHOL, i, m))              # L_im and L_ii^{-1}
        for m in range(i):
            p0.add((LSOLVE, m, j))            # X tiles above
    elif ty == RSOLVE:
        for col in (j, T + j):
            for k in range(T):
                p0.add((LSOLVE, k, col))      # X_ij ready; every reader of X_ij done
        for m in range(j):
            p0.add((RSOLVE, i, m))            # W_im
        for m in range(j + 1):
            p0.add((CHOL, j, m))              # L_jm, L_jj^{-1}
    elif ty == REDUCE:
        p0 = {t for t in expected_tasks(T, mode) if t[0] != REDUCE}
    return p0, p1


def _fields(ns, modes, bt):
    return [(_tiles(n, bt), m) for n, m in zip(ns, modes)]


CASES = [
    ([1], [2], 64),
    ([63], [2], 64),            # n + 1 = 64: one tile
    ([64], [2], 64),            # the border row starts a second tile
    ([200, 127, 5], [2, 1, 2], 64),
    ([300, 40, 129], [1, 2, 0], 128),
    ([500, 257, 90, 1000], [2, 2, 1, 2], 128),
]


@pytest.mark.parametrize("ns,modes,bt", CASES)
@pytest.mark.parametrize("slots,queues", [(1, 1), (7, 1), (512, 1), (16, 2), (512, 8)])
def test_ticket_order_complete_and_ordered(ns, modes, bt, slots, queues):
    order, qoff, est = fbt.round_plan(ns, modes, tile=bt, slots=slots, queues=queues)
    assert est > 0 and qoff[0] == 0 and qoff[-1] == len(order) and np.all(np.diff(qoff) >= 0)
    fl = _fields(ns, modes, bt)
    seen, queue = {}, {}
    for q, (f, ty, i, j) in enumerate(order.tolist()):
        key = (f, ty, i, j)
        assert key not in seen, key
        seen[key] = q
        qq = int(np.searchsorted(qoff, q, side="right")) - 1
        assert queue.setdefault(f, qq) == qq, "a field's tasks span two queues"
    for f, (T, m) in enumerate(fl):
        got = {(ty, i, j) for (ff, ty, i, j) in seen if ff == f}
        assert got == expected_tasks(T, m), f
    for (f, ty, i, j), q in seen.items():
        T, m = fl[f]
        p0, p1 = predecessors((ty, i, j), T, m)
        for p in p0 | p1:
            assert seen[(f,) + p] < q, ((f, ty, i, j), p)


def _simulate(order, fl, workers, rng, qoff=None, task_deps=None):
    """Random interleaving of `workers` workgroups taking tickets in order and
    waiting on the kernel's counters (with queues: worker w takes tickets of
    queue w % len(queues) only); checks the true predecessors at every start
    of a phase.  Returns the number of finished tasks."""
    if qoff is None:
        qoff = [0, len(order)]
    task_deps = task_deps or fbt.round_task_deps
    nq = len(qoff) - 1
    nxt_q = list(qoff[:-1])
    cnt = [dict() for _ in fl]
    deps = {}

    def dep(f, ty, i, j):
        key = (f, ty, i, j)
        if key not in deps:
            T, m = fl[f]
            deps[key] = task_deps(T, m, f, ty, i, j)
        return deps[key]

    done = set()
    state = [None] * workers      # None idle, else [task, stage]
    # stages: 0 waiting (first waits), 1 running phase 0, 2 waiting (last wait), 3 running phase 1
    while True:
        actions = []
        for w in range(workers):
            st = state[w]
            if st is None:
                if nxt_q[w % nq] < qoff[w % nq + 1]:
                    actions.append((w, "take"))
                continue
            (f, ty, i, j), stage = st
            waits, _ = dep(f, ty, i, j)
            split = ty == CHOL and i > j
            first = waits[:-1] if split else waits
            if stage == 0 and all(cnt[f].get(o, 0) >= v for o, v in first):
                actions.append((w, "start"))
            elif stage in (1, 3):
                actions.append((w, "finish"))
            elif stage == 2 and all(cnt[f].get(o, 0) >= v for o, v in waits[-1:]):
                actions.append((w, "start1"))
        if not actions:
            break
        w, act = rng.choice(actions)
        if act == "take":
            state[w] = [tuple(order[nxt_q[w % nq]]), 0]
            nxt_q[w % nq] += 1
            continue
        (f, ty, i, j), stage = state[w]
        T, m = fl[f]
        p0, p1 = predecessors((ty, i, j), T, m)
        if act == "start":
            for p in p0:
                assert (f,) + p in done, ((f, ty, i, j), p)
            state[w][1] = 1
        elif act == "start1":
            for p in p1:
                assert (f,) + p in done, ((f, ty, i, j), p)
            state[w][1] = 3
        else:  # finish
            if ty == CHOL and i > j and stage == 1:
                state[w][1] = 2
                continue
            _, pub = dep(f, ty, i, j)
            for o in pub:
                cnt[f][o] = cnt[f].get(o, 0) + 1
            done.add((f, ty, i, j))
            state[w] = None
    return len(done)


@pytest.mark.parametrize("ns,modes,bt", CASES[:5])
def test_counter_waits_imply_data_order(ns, modes, bt):
    rng = random.Random(1234)
    fl = _fields(ns, modes, bt)
    for slots, workers, queues in ((1, 1, 1), (7, 3, 1), (512, 8, 1), (512, 600, 1),
                                   (16, 4, 2), (512, 16, 8), (512, 64, 8)):
        order, qoff, _ = fbt.round_plan(ns, modes, tile=bt, slots=slots, queues=queues)
        for rep in range(3):
            finished = _simulate(order.tolist(), fl, workers, rng, qoff.tolist())
            assert finished == len(order), (slots, workers, queues, rep)


def test_plan_rejects_bad_arguments():
    with pytest.raises(fbt.FisherBTError):
        fbt.round_plan([100], [2], tile=96)
    with pytest.raises(fbt.FisherBTError):
        fbt.round_plan([0], [2], tile=64)
    with pytest.raises(fbt.FisherBTError):
        fbt.round_plan([10], [2], tile=64, queues=9)
    order, _, _ = fbt.round_plan([100, 50], [0, 3], tile=64)
    assert len(order) == 0


def test_plan_of_the_many_field_round():
    """256 fields, n ~ U[500, 4000] (the batched workload): the plan is built
    and checked on the host for one queue and for one per XCD."""
    rng = np.random.default_rng(5)
    ns = rng.integers(500, 4001, size=256)
    for bt, slots in ((64, 512), (128, 256)):
        T = [(n + 1 + bt - 1) // bt for n in ns]
        for queues in (1, 8):
            order, qoff, est = fbt.round_plan(ns, [2] * 256, tile=bt, slots=slots, queues=queues)
            assert len(order) == sum(3 * t * (t + 1) // 2 + 2 * t * t + 1 for t in T)
            assert est > 0


MUTATIONS = {
    # a forward-substitution tile waits for one X tile too few above it
    "lsolve_one_short": ("off[k] = c.xd + j, need[k++] = i; // X tiles above",
                         "off[k] = c.xd + j, need[k++] = i - 1; // X tiles above"),
    # a W tile does not wait for the nu-matrix column of X
    "rsolve_no_nu_column": ("        off[k] = c.xd + T + j, need[k++] = T;\n", ""),
    # a Cholesky tile takes the previous block column as finished one tile early
    "chol_column_early": ("need[k++] = T - j + 1; // block columns",
                          "need[k++] = T - j; // block columns"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_counter_mistakes_are_caught(name, tmp_path):
    """The counter waits of the kernel with one mistake planted (a copy of
    the header, compiled on the host with the planner): the random
    interleavings must then run some task before its data are ready."""
    import ctypes
    import os
    import shutil
    import subprocess

    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    csrc = os.path.join(root, "paper_2601_11437_amd", "csrc")
    hdr = open(os.path.join(csrc, "fbt_round.h")).read()
    old, new = MUTATIONS[name]
    assert old in hdr
    (tmp_path / "fbt_round.h").write_text(hdr.replace(old, new))
    # the planner's sources beside the planted header, so that their quoted
    # includes find it
    for src in ("fbt_plan.h", "fbt_plan.cpp"):
        shutil.copy(os.path.join(csrc, src), tmp_path / src)
    so = str(tmp_path / "libplan.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I",
                    os.path.join(root, "include"), str(tmp_path / "fbt_plan.cpp"), "-o", so],
                   check=True, capture_output=True)
    L = ctypes.CDLL(so)
    f = L.fbt_round_task_deps
    f.restype, f.argtypes = fbt.SIGNATURES["fbt_round_task_deps"]
    # the planted copy differs from the library's waits
    probe = {"lsolve_one_short": (8, 2, 2, 5, 3), "rsolve_no_nu_column": (8, 2, 3, 5, 3),
             "chol_column_early": (8, 2, 1, 5, 3)}[name]

    def deps(T, mode, field, type_, i, j):
        off, need, pub = (np.zeros(4, dtype=np.int32) for _ in range(3))
        npub = ctypes.c_int32(0)
        k = f(T, mode, (field << 3) | type_, (i << 16) | j, off.ctypes.data, need.ctypes.data,
              pub.ctypes.data, ctypes.byref(npub))
        return list(zip(off[:k].tolist(), need[:k].tolist())), pub[:npub.value].tolist()

    T_, m_, ty_, i_, j_ = probe
    assert deps(T_, m_, 0, ty_, i_, j_) != fbt.round_task_deps(T_, m_, 0, ty_, i_, j_)
    rng = random.Random(7)
    caught = False
    for ns, modes, bt in CASES:
        fl = _fields(ns, modes, bt)
        for slots, workers in ((7, 3), (512, 8), (512, 600)):
            order, qoff, _ = fbt.round_plan(ns, modes, tile=bt, slots=slots, queues=1)
            for rep in range(3):
                try:
                    _simulate(order.tolist(), fl, workers, rng, qoff.tolist(), task_deps=deps)
                except AssertionError:
                    caught = True
                    break
            if caught:
                break
        if caught:
            break
    assert caught, name
