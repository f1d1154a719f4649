"""Host-side checks of the C ABI (no GPU): every declared symbol is exported,
the L9 design of Table 1, argument errors, and the Fisher-BT driver
(Algorithm 1) of the library against the oracle's driver on the same
evaluators."""
import ctypes
import json
import math
import os
import re

import numpy as np
import pytest

import paper_2601_11437_amd as fbt
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fisherbt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fbt_\w+)\s*\((?!\s*\*)", src)))


def test_library_exports_every_declared_symbol():
    L = fbt.lib()
    names = _declared()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), name
        assert name in fbt.SIGNATURES, name


def test_status_strings():
    L = fbt.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.fbt_status_string(code)
    assert L.fbt_status_string(123) == b"unknown status"


def test_null_arguments_are_rejected():
    L = fbt.lib()
    th = np.array([1.0, 0.1, 0.5])
    assert L.fbt_loglik(None, th.ctypes.data, th.ctypes.data) == fbt.EINVAL
    assert L.fbt_eval(None, th.ctypes.data, None, None, None) == fbt.EINVAL
    # pointers as the binding passes them (c_void_p), for the adjoint entry point
    out = np.zeros(4)
    assert L.fbt_grad(None, fbt._ptr(th), fbt._ptr(out), fbt._ptr(out[1:]), None) == fbt.EINVAL
    assert L.fbt_create(None, None) == fbt.EINVAL
    assert L.fbt_fit_evaluator(None, None, None) == fbt.EINVAL
    assert L.fbt_set_timing(None, 1) == fbt.EINVAL
    assert L.fbt_set_sigma_nu_mode(None, 0) == fbt.EINVAL
    assert L.fbt_set_wphase(None, fbt.WPHASE_TWO_SIDED) == fbt.EINVAL
    assert L.fbt_set_refinement(None, 2) == fbt.EINVAL
    assert L.fbt_set_precision(None, 0) == fbt.EINVAL
    assert (fbt.FP64, fbt.MIXED_FP32, fbt.MIXED_FP32_ALL, fbt.MIXED_BF16,
            fbt.MIXED_BF16_ALL) == (0, 1, 2, 3, 4)
    L.fbt_destroy(None)                      # NULL-safe
    # batch entry points
    cfg = fbt.Config(0, 0, 0, None)
    assert L.fbt_batch_create(None, 1, None) == fbt.EINVAL
    assert L.fbt_batch_create(ctypes.byref(cfg), 0, ctypes.byref(ctypes.c_void_p())) == fbt.EINVAL
    assert L.fbt_batch_set_fields(None, 0, None, None, None) == fbt.EINVAL
    assert L.fbt_batch_eval(None, None, None, None, None, None, None) == fbt.EINVAL
    assert L.fbt_batch_set_exec(None, 0) == fbt.EINVAL
    assert L.fbt_batch_get_exec(None) == -1
    assert L.fbt_batch_set_group_limit(None, 256, 1) == fbt.EINVAL
    assert L.fbt_batch_group_limit(None, 256) == -1
    assert L.fbt_batch_autotune(None, None, None, None) == fbt.EINVAL
    assert L.fbt_batch_load_tuning(None, b"x.json") == fbt.EINVAL
    L.fbt_batch_destroy(None)                # NULL-safe
    # allocation-free entry point: every argument error is caught before the
    # device is touched (host memory stands in for the device arrays)
    locs, z = np.zeros((8, 2)), np.zeros(8)
    ll, sc, fi = np.zeros(1), np.zeros(3), np.zeros(9)
    ptrs = [fbt._ptr(a) for a in (locs, z, th, ll, sc, fi)]
    na = L.fbt_eval_noalloc
    assert na(0, None, 8, None, *ptrs[1:]) == fbt.EINVAL
    assert na(0, None, 0, *ptrs) == fbt.EINVAL
    assert na(0, None, 1024, *ptrs) == fbt.EINVAL                    # above the maximum n
    assert na(16, None, 8, *ptrs) == fbt.EINVAL
    bad = np.array([1.0, -0.1, 0.5])
    assert na(0, None, 8, ptrs[0], ptrs[1], fbt._ptr(bad), *ptrs[3:]) == fbt.EINVAL
    assert na(0, None, 8, *ptrs[:5], None) == fbt.EINVAL


def test_batch_create_without_gpu_fails_cleanly():
    try:
        import torch

        if torch.cuda.device_count() > 0:
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    L = fbt.lib()
    cfg = fbt.Config(0, 0, 0, None)
    h = ctypes.c_void_p()
    assert L.fbt_batch_create(ctypes.byref(cfg), 2, ctypes.byref(h)) == fbt.EDEVICE
    assert not h.value


def test_l9_design_matches_table1():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "table1_l9.json")))
    lo, hi = g["simulation_bounds"]["lower"], g["simulation_bounds"]["upper"]
    want = np.array([[g["levels"][c][0] * lo[k] + g["levels"][c][1] * hi[k]
                      for k, c in enumerate(row)] for row in g["rows"]])
    np.testing.assert_allclose(fbt.l9_design(lo, hi), want, rtol=1e-15)
    np.testing.assert_allclose(fbt.l9_design(lo, hi)[0], g["candidate_1_at_simulation_bounds"],
                               rtol=1e-15)


class Quadratic:
    def __init__(self, m, H, scale=1.0, valid=lambda t: True):
        self.m, self.H, self.k, self.valid = np.asarray(m, float), np.asarray(H, float), scale, valid

    def loglik(self, t):
        t = np.asarray(t, float)
        if not self.valid(t):
            return -math.inf
        d = t - self.m
        return float(-0.5 * d @ self.H @ d)

    def lib_loglik(self, t):
        v = self.loglik(t)
        if v == -math.inf:
            raise ArithmeticError
        return v

    def evaluate(self, t):
        d = np.asarray(t, float) - self.m
        return float(-0.5 * d @ self.H @ d), -self.H @ d, self.k * self.H


H = np.array([[2.0, 0.3, 0.1], [0.3, 1.0, 0.2], [0.1, 0.2, 0.5]])
CASES = [
    dict(m=[1.0, 0.5, 0.7], scale=1.0, theta0=[3.0, 2.0, 1.5], kw={}),
    dict(m=[1.0, 0.5, 0.7], scale=1 / 3, theta0=[1.3, 0.6, 0.8], kw=dict(max_iter=1, nelder_mead=0)),
    dict(m=[1.0, 0.5, 0.7], scale=1 / 8, theta0=[1.3, 0.6, 0.8], kw=dict(nelder_mead=0)),
    dict(m=[0.2, 0.5, 0.7], scale=1 / 3, theta0=[0.6, 0.6, 0.8], kw=dict(max_iter=1, nelder_mead=0)),
    dict(m=[1.0, 0.5, 0.7], scale=1000.0, theta0=[1.5, 0.9, 1.1], kw={}),
    dict(m=[1.0, 0.5, 0.7], scale=1e-6, theta0=[1.5, 0.9, 1.1], kw=dict(nelder_mead=0)),
    dict(m=[2.505, 2.505, 1.005], scale=1.0, theta0=None, kw={}),
]


@pytest.mark.parametrize("case", CASES)
def test_driver_matches_oracle_driver_on_mock(oracle_mod, case):
    q = Quadratic(case["m"], H, case["scale"], valid=lambda t: np.all(t > 0))
    kw = dict(case["kw"])
    got = fbt.fit_with(q.lib_loglik, q.evaluate, theta0=case["theta0"], **kw)
    okw = {"max_iter": kw.get("max_iter", 0), "use_nelder_mead": bool(kw.get("nelder_mead", 1))}
    want = oracle_mod.fisher_bt(q, theta0=case["theta0"], **okw)
    assert got["converged"] == want["converged"]
    assert got["used_nelder_mead"] == want["used_nelder_mead"]
    for k in ("n_loglik_calls", "n_grad_calls", "n_iter"):
        assert got[k] == want[k], k
    np.testing.assert_allclose(got["theta"], want["theta"], rtol=1e-12, atol=1e-14)
    if not want["converged"] and not want["used_nelder_mead"]:
        assert got["status"] == fbt.EBUDGET


def test_driver_matches_oracle_driver_on_matern(oracle_mod):
    """Same oracle evaluations, two independent drivers: same path and result."""
    locs, z, _ = synth.dataset(150, (1.0, 0.1, 0.5), 77)
    ev = oracle_mod.OracleEvaluator(locs, z)

    def ll(t):
        v = ev.loglik(t)
        if v == -math.inf:
            raise ArithmeticError
        return v

    seen = []
    got = fbt.fit_with(ll, ev.evaluate, theta0=(0.5, 0.05, 1.0), max_iter=50,
                       callback=lambda it, th, l, g, f: seen.append(th))
    want = oracle_mod.fisher_bt(ev, theta0=(0.5, 0.05, 1.0), max_iter=50)
    assert got["converged"] and want["converged"]
    assert (got["n_loglik_calls"], got["n_grad_calls"]) == (want["n_loglik_calls"], want["n_grad_calls"])
    np.testing.assert_allclose(got["theta"], want["theta"], rtol=1e-9)
    assert len(seen) == got["n_iter"] + 1
    # precision switching belongs to the GPU evaluator of fbt_fit only
    assert got["precision_switch"] == -1 and got["n_fp64_evals"] == 0


def test_fit_option_defaults():
    """fbt_fit_options_default: the paper's constants (Section 2.1, Eq. (4))
    and the mixed-precision switch point."""
    o, _ = fbt._options()
    assert tuple(o.lo) == (0.01, 0.01, 0.01) and tuple(o.hi) == (5.0, 5.0, 2.0)
    assert (o.armijo_c, o.armijo_relax, o.backtrack_rho, o.grad_tol) == (1e-3, 1e-3, 0.5, 1e-3)
    assert (o.max_loglik_calls, o.max_grad_calls, o.max_iter, o.nelder_mead) == (60, 20, 0, 1)
    assert (o.nm_ftol, o.nm_max_evals) == (1e-9, 500)
    assert o.mixed_switch == 1e-4


def test_create_without_gpu_fails_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(fbt.FisherBTError) as e:
        fbt.Context(0)
    assert e.value.status == fbt.EDEVICE
