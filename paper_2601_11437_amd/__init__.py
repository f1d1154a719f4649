"""Python binding of libfisherbt (C ABI in include/fisherbt.h).

Exact Matern maximum likelihood by Fisher scoring with backtracking
(Fisher-BT): log-likelihood (Algorithm 2), score and Fisher information
(Algorithm 3) and the fit (Algorithm 1), all evaluated by HIP kernels on an
MI355X.  This module only marshals arguments; every step of an evaluation runs
in the library.  It raises if the library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfisherbt.so")

OK, EINVAL, ENOTPD, ENOMEM, EDEVICE, ENONFINITE, EBUDGET, ENODATA = 0, -1, -2, -3, -4, -5, -6, -7

# kernel classes of fbt_get_timing
KERNEL_CLASSES = ("generation", "diag_factor_inverse", "panel_solve", "cholesky_update",
                  "left_diag_apply", "left_update", "right_panel_reduce", "right_update",
                  "reductions", "adjoint_inverse", "adjoint_xtx", "adjoint_contraction",
                  "twosided_diag", "twosided_panel", "twosided_update", "deferred_diag_apply",
                  "deferred_update", "twosided_lookahead")

_lib = None
_d = ctypes.c_double
_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)

LOGLIK_FN = ctypes.CFUNCTYPE(ctypes.c_int, _p, _dp, _dp)
EVAL_FN = ctypes.CFUNCTYPE(ctypes.c_int, _p, _dp, _dp, _dp, _dp)
ITER_CB = ctypes.CFUNCTYPE(None, _p, _i32, _dp, _d, _dp, _dp)


class FitOptions(ctypes.Structure):
    _fields_ = [("theta0", _dp), ("lo", _d * 3), ("hi", _d * 3), ("armijo_c", _d),
                ("armijo_relax", _d), ("backtrack_rho", _d), ("grad_tol", _d),
                ("max_loglik_calls", _i32), ("max_grad_calls", _i32), ("max_iter", _i32),
                ("nelder_mead", _i32), ("nm_ftol", _d), ("nm_max_evals", _i32),
                ("cb", ITER_CB), ("cb_user", _p), ("mixed_switch", _d)]


class FitResult(ctypes.Structure):
    _fields_ = [("theta", _d * 3), ("loglik", _d), ("score", _d * 3), ("fisher", _d * 9),
                ("n_loglik_calls", _i32), ("n_grad_calls", _i32), ("n_iter", _i32),
                ("used_nelder_mead", _i32), ("converged", _i32), ("n_nm_evals", _i32),
                ("n_fp64_evals", _i32), ("precision_switch", _i32)]


class Config(ctypes.Structure):
    _fields_ = [("device", _i32), ("tile", _i32), ("precision", _i32), ("hip_stream", _p)]


FP64, MIXED_FP32, MIXED_FP32_ALL, MIXED_BF16, MIXED_BF16_ALL = 0, 1, 2, 3, 4
SIGMA_NU_EXACT, SIGMA_NU_PAPER = 0, 1
WPHASE_TWO_SIDED, WPHASE_SOLVES = 0, 1


class Evaluator(ctypes.Structure):
    _fields_ = [("user", _p), ("loglik", LOGLIK_FN), ("eval", EVAL_FN)]


# name -> (restype, argtypes): every symbol the header declares
SIGNATURES = {
    "fbt_create": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(_p)]),
    "fbt_destroy": (None, [_p]),
    "fbt_set_precision": (ctypes.c_int, [_p, _i32]),
    "fbt_set_data": (ctypes.c_int, [_p, _i64, _p, _p]),
    "fbt_set_data_device": (ctypes.c_int, [_p, _i64, _p, _p]),
    "fbt_loglik": (ctypes.c_int, [_p, _p, _p]),
    "fbt_eval": (ctypes.c_int, [_p, _p, _p, _p, _p]),
    "fbt_eval_terms": (ctypes.c_int, [_p, _p, _p]),
    "fbt_covariance": (ctypes.c_int, [_p, _p, _i32, _p, _i64]),
    "fbt_factor": (ctypes.c_int, [_p, _p, _p, _i64]),
    "fbt_fit_options_default": (None, [ctypes.POINTER(FitOptions)]),
    "fbt_fit": (ctypes.c_int, [_p, ctypes.POINTER(FitOptions), ctypes.POINTER(FitResult)]),
    "fbt_fit_evaluator": (ctypes.c_int, [ctypes.POINTER(Evaluator), ctypes.POINTER(FitOptions),
                                         ctypes.POINTER(FitResult)]),
    "fbt_l9_design": (None, [_p, _p, _p]),
    "fbt_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "fbt_last_error": (ctypes.c_char_p, [_p]),
    "fbt_last_notpd_pivot": (_i64, [_p]),
    "fbt_grad": (ctypes.c_int, [_p, _p, _p, _p, _p]),
    "fbt_set_sigma_nu_mode": (ctypes.c_int, [_p, _i32]),
    "fbt_set_wphase": (ctypes.c_int, [_p, _i32]),
    "fbt_set_refinement": (ctypes.c_int, [_p, _i32]),
    "fbt_eval_noalloc": (ctypes.c_int, [_i32, _p, _i64, _p, _p, _p, _p, _p, _p]),
    "fbt_batch_create": (ctypes.c_int, [ctypes.POINTER(Config), _i32, ctypes.POINTER(_p)]),
    "fbt_batch_destroy": (None, [_p]),
    "fbt_batch_set_fields": (ctypes.c_int, [_p, _i32, _p, _p, _p]),
    "fbt_batch_eval": (ctypes.c_int, [_p, _p, _p, _p, _p, _p, _p]),
    "fbt_batch_last_error": (ctypes.c_char_p, [_p]),
    "fbt_batch_set_exec": (ctypes.c_int, [_p, _i32]),
    "fbt_batch_get_exec": (_i32, [_p]),
    "fbt_batch_set_group_limit": (ctypes.c_int, [_p, _i64, _i32]),
    "fbt_batch_group_limit": (_i32, [_p, _i64]),
    "fbt_batch_autotune": (ctypes.c_int, [_p, _p, _p, ctypes.c_char_p]),
    "fbt_batch_load_tuning": (ctypes.c_int, [_p, ctypes.c_char_p]),
    "fbt_batch_fit": (ctypes.c_int, [_p, ctypes.POINTER(FitOptions), _p, _p, _p, _p,
                                     ctypes.POINTER(_i32)]),
    "fbt_batch_set_fit_threads": (ctypes.c_int, [_p, _i32]),
    "fbt_batch_set_tile": (ctypes.c_int, [_p, _i32]),
    "fbt_batch_get_tile": (_i32, [_p]),
    "fbt_batch_round_stats": (ctypes.c_int, [_p, ctypes.POINTER(_i64), _dp, _dp]),
    "fbt_batch_set_round_trace": (ctypes.c_int, [_p, _i32]),
    "fbt_batch_set_round_graph": (ctypes.c_int, [_p, _i32]),
    "fbt_batch_round_trace": (_i64, [_p, _p, _i64]),
    "fbt_round_plan": (ctypes.c_int, [_i32, _p, _p, _i32, _i32, _i32, ctypes.POINTER(_i64), _p,
                                      _p, _dp]),
    "fbt_batch_set_queues": (ctypes.c_int, [_p, _i32]),
    "fbt_batch_get_queues": (_i32, [_p]),
    "fbt_round_task_deps": (_i32, [_i32, _i32, _i32, _i32, _p, _p, _p, ctypes.POINTER(_i32)]),
    "fbt_set_timing": (ctypes.c_int, [_p, _i32]),
    "fbt_get_timing": (ctypes.c_int, [_p, _i32, ctypes.POINTER(_i64), _dp, _dp]),
}


def _share_torch_hip_runtime():
    """PyTorch ships its own HIP runtime with the same soname as the system one.
    Two runtimes in one process cannot both open the GPU, so when PyTorch is
    installed its copy is loaded first and libfisherbt binds to it."""
    import importlib.util

    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        return
    path = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
    if os.path.exists(path):
        ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)


def lib() -> ctypes.CDLL:
    """Load libfisherbt.so (built by ``paper_2601_11437_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfisherbt.so is not built; run `python -m paper_2601_11437_amd.build`")
        _share_torch_hip_runtime()
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class FisherBTError(RuntimeError):
    def __init__(self, status: int, detail: str = "", pivot: int = -1):
        self.status = status
        self.pivot = pivot
        msg = lib().fbt_status_string(status).decode()
        super().__init__("%s (%d)%s" % (msg, status, (": " + detail) if detail else ""))


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError("expected %d values" % n)
    return a


def _ptr(a):
    return a.ctypes.data_as(_p)


def l9_design(lo, hi) -> np.ndarray:
    """The nine starting candidates of Table 1 (9 x 3)."""
    lo, hi = _arr(lo, 3), _arr(hi, 3)
    out = np.empty(27)
    lib().fbt_l9_design(_ptr(lo), _ptr(hi), _ptr(out))
    return out.reshape(9, 3)


def _options(theta0=None, lo=None, hi=None, callback=None, **kw):
    o = FitOptions()
    lib().fbt_fit_options_default(ctypes.byref(o))
    keep = []
    if theta0 is not None:
        t0 = (_d * 3)(*[float(v) for v in theta0])
        keep.append(t0)
        o.theta0 = ctypes.cast(t0, _dp)
    if lo is not None:
        o.lo = (_d * 3)(*[float(v) for v in lo])
    if hi is not None:
        o.hi = (_d * 3)(*[float(v) for v in hi])
    for k, v in kw.items():
        if not hasattr(o, k) or k in ("theta0", "cb", "cb_user"):
            raise TypeError("unknown fit option %r" % k)
        setattr(o, k, v)
    if callback is not None:
        def _cb(user, it, th, ll, sc, fi):
            callback(int(it), np.array(th[:3]), float(ll), np.array(sc[:3]),
                     np.array(fi[:9]).reshape(3, 3))
        cb = ITER_CB(_cb)
        keep.append(cb)
        o.cb = cb
    return o, keep


def _result(r: FitResult) -> dict:
    return {"theta": np.array(r.theta[:]), "loglik": r.loglik, "score": np.array(r.score[:]),
            "fisher": np.array(r.fisher[:]).reshape(3, 3), "n_loglik_calls": r.n_loglik_calls,
            "n_grad_calls": r.n_grad_calls, "n_iter": r.n_iter,
            "used_nelder_mead": bool(r.used_nelder_mead), "converged": bool(r.converged),
            "n_nm_evals": r.n_nm_evals, "n_fp64_evals": r.n_fp64_evals,
            "precision_switch": r.precision_switch}


def fit_with(loglik, evaluate, **opts) -> dict:
    """Algorithm 1 (the library's driver) over Python callables:
    loglik(theta) -> float (raise ArithmeticError for a non-positive-definite
    covariance) and evaluate(theta) -> (l, grad[3], fisher[3, 3])."""
    def _ll(user, th, out):
        try:
            out[0] = float(loglik(np.array(th[:3])))
            return OK
        except ArithmeticError:
            return ENOTPD

    def _ev(user, th, ll, sc, fi):
        try:
            v, g, f = evaluate(np.array(th[:3]))
        except ArithmeticError:
            return ENOTPD
        ll[0] = float(v)
        for i in range(3):
            sc[i] = float(g[i])
        f = np.asarray(f, dtype=np.float64).ravel()
        for i in range(9):
            fi[i] = float(f[i])
        return OK

    ev = Evaluator(None, LOGLIK_FN(_ll), EVAL_FN(_ev))
    o, keep = _options(**opts)
    r = FitResult()
    st = lib().fbt_fit_evaluator(ctypes.byref(ev), ctypes.byref(o), ctypes.byref(r))
    if st not in (OK, EBUDGET):
        raise FisherBTError(st)
    out = _result(r)
    out["status"] = st
    return out


class Context:
    """One device context: data on the GPU and the evaluation calls."""

    def __init__(self, device: int = 0, stream=None, precision: int = FP64):
        cfg = Config(int(device), 0, int(precision), None)
        if stream is not None:
            cfg.hip_stream = int(getattr(stream, "cuda_stream", stream))
        h = _p()
        st = lib().fbt_create(ctypes.byref(cfg), ctypes.byref(h))
        if st != OK:
            raise FisherBTError(st, "fbt_create(device=%d)" % device)
        self._h = h
        self.n = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().fbt_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st != OK:
            L = lib()
            raise FisherBTError(st, L.fbt_last_error(self._h).decode(),
                                int(L.fbt_last_notpd_pivot(self._h)))

    def set_data(self, locs, z):
        """Locations (n x 2) and observations (n): numpy arrays, or torch tensors
        (device tensors are passed by pointer)."""
        if hasattr(locs, "is_cuda") and locs.is_cuda:
            import torch

            lt = locs.detach().to(torch.float64).contiguous()
            zt = z.detach().to(device=lt.device, dtype=torch.float64).contiguous()
            torch.cuda.current_stream(lt.device).synchronize()   # producer stream -> library stream
            n = int(zt.numel())
            if lt.numel() != 2 * n:
                raise ValueError("locs must be n x 2")
            self._check(lib().fbt_set_data_device(self._h, n, _p(lt.data_ptr()), _p(zt.data_ptr())))
        else:
            locs = _arr(np.asarray(locs.cpu() if hasattr(locs, "cpu") else locs))
            z = _arr(np.asarray(z.cpu() if hasattr(z, "cpu") else z))
            n = z.size
            if locs.size != 2 * n:
                raise ValueError("locs must be n x 2")
            self._check(lib().fbt_set_data(self._h, n, _ptr(locs), _ptr(z)))
        self.n = n

    def loglik(self, theta) -> float:
        th = _arr(theta, 3)
        out = np.zeros(1)
        self._check(lib().fbt_loglik(self._h, _ptr(th), _ptr(out)))
        return float(out[0])

    def eval(self, theta):
        """(loglik, score[3], fisher[3, 3]) by Algorithm 3."""
        th = _arr(theta, 3)
        ll, sc, fi = np.zeros(1), np.zeros(3), np.zeros(9)
        self._check(lib().fbt_eval(self._h, _ptr(th), _ptr(ll), _ptr(sc), _ptr(fi)))
        return float(ll[0]), sc, fi.reshape(3, 3)

    def grad(self, theta, dz: bool = False):
        """(loglik, score[3]) by the adjoint form of Eq. (2), no Fisher
        information; with dz=True also dl/dZ (n,) as a third element."""
        th = _arr(theta, 3)
        ll, sc = np.zeros(1), np.zeros(3)
        g = np.zeros(self.n) if dz else None
        self._check(lib().fbt_grad(self._h, _ptr(th), _ptr(ll), _ptr(sc),
                                   _ptr(g) if dz else None))
        return (float(ll[0]), sc, g) if dz else (float(ll[0]), sc)

    def eval_terms(self, theta) -> np.ndarray:
        th = _arr(theta, 3)
        t = np.zeros(9)
        self._check(lib().fbt_eval_terms(self._h, _ptr(th), _ptr(t)))
        return t

    def covariance(self, theta, which: int = 0) -> np.ndarray:
        th = _arr(theta, 3)
        out = np.empty((self.n, self.n), order="F")
        self._check(lib().fbt_covariance(self._h, _ptr(th), int(which), _ptr(out), self.n))
        return out

    def factor(self, theta) -> np.ndarray:
        th = _arr(theta, 3)
        out = np.empty((self.n, self.n), order="F")
        self._check(lib().fbt_factor(self._h, _ptr(th), _ptr(out), self.n))
        return out

    def fit(self, **opts) -> dict:
        o, keep = _options(**opts)
        r = FitResult()
        st = lib().fbt_fit(self._h, ctypes.byref(o), ctypes.byref(r))
        if st not in (OK, EBUDGET):
            self._check(st)
        out = _result(r)
        out["status"] = st
        return out

    def set_precision(self, precision: int):
        """FP64 (0), MIXED_FP32 (1: solve updates in FP32), MIXED_FP32_ALL
        (2: Cholesky updates too), MIXED_BF16 (3: solve updates with
        bfloat16 operands and FP32 sums) or MIXED_BF16_ALL (4: Cholesky
        updates too) for the following evaluations."""
        self._check(lib().fbt_set_precision(self._h, int(precision)))

    def set_sigma_nu_mode(self, mode: int):
        """SIGMA_NU_EXACT (0, default) or SIGMA_NU_PAPER (1: the case scheme of
        Supplementary A for dSigma/dnu)."""
        self._check(lib().fbt_set_sigma_nu_mode(self._h, int(mode)))

    def set_wphase(self, form: int):
        """WPHASE_TWO_SIDED (0, default: blocked two-sided reduction, n^3 flops
        per derivative matrix, FP64) or WPHASE_SOLVES (1: left block solve and
        lower-half right solve, 4 n^3 / 3 per matrix; the mixed precisions
        always take it) for the W phase of the following evaluations."""
        self._check(lib().fbt_set_wphase(self._h, int(form)))

    def set_refinement(self, iterations: int):
        """Refinement steps of w = Sigma^{-1} Z under MIXED_FP32_ALL (default
        0: off)."""
        self._check(lib().fbt_set_refinement(self._h, int(iterations)))

    def set_timing(self, enable: bool):
        self._check(lib().fbt_set_timing(self._h, 1 if enable else 0))

    def timing(self) -> dict:
        out = {}
        for k, name in enumerate(KERNEL_CLASSES):
            n, ms, fl = _i64(), _d(), _d()
            self._check(lib().fbt_get_timing(self._h, k, ctypes.byref(n), ctypes.byref(ms),
                                             ctypes.byref(fl)))
            out[name] = {"launches": n.value, "ms": ms.value, "flops": fl.value}
        return out


class Batch:
    """Many independent fields evaluated together (fbt_batch_*): a pool of
    `workers` device contexts fed by host threads, longest field first, or one
    HIP graph per call (exec GRAPH); group sizes per padded order from
    set_group_limit or the autotuner."""

    SKIP, LOGLIK, EVAL, GRAD = 0, 1, 2, 3
    WORKERS, GRAPH, PERSISTENT = 0, 1, 2

    def __init__(self, workers: int = 2, device: int = 0, precision: int = FP64):
        cfg = Config(int(device), 0, int(precision), None)
        h = _p()
        st = lib().fbt_batch_create(ctypes.byref(cfg), int(workers), ctypes.byref(h))
        if st != OK:
            raise FisherBTError(st, "fbt_batch_create(workers=%d)" % workers)
        self._h = h
        self.nf = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().fbt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_fields(self, fields):
        """fields: sequence of (locs (n x 2), z (n)) numpy pairs."""
        locs = [np.ascontiguousarray(l, dtype=np.float64) for l, _ in fields]
        zs = [np.ascontiguousarray(z, dtype=np.float64) for _, z in fields]
        n = np.array([z.size for z in zs], dtype=np.int64)
        lp = (_p * len(locs))(*[a.ctypes.data for a in locs])
        zp = (_p * len(zs))(*[a.ctypes.data for a in zs])
        st = lib().fbt_batch_set_fields(self._h, len(zs), n.ctypes.data, lp, zp)
        if st != OK:
            raise FisherBTError(st, "fbt_batch_set_fields")
        self._keep = (locs, zs)
        self.nf = len(zs)

    def eval(self, thetas, mode):
        """thetas (nf x 3), mode (nf,) in {SKIP, LOGLIK, EVAL, GRAD}.
        Returns (loglik (nf,), score (nf, 3), fisher (nf, 3, 3), status (nf,));
        entries of fields that were skipped or failed are NaN."""
        th = np.ascontiguousarray(thetas, dtype=np.float64).reshape(self.nf, 3)
        md = np.ascontiguousarray(np.broadcast_to(np.asarray(mode, dtype=np.int32), (self.nf,)))
        ll = np.full(self.nf, np.nan)
        sc = np.full((self.nf, 3), np.nan)
        fi = np.full((self.nf, 9), np.nan)
        status = np.zeros(self.nf, dtype=np.int32)
        st = lib().fbt_batch_eval(self._h, th.ctypes.data, md.ctypes.data, ll.ctypes.data,
                                  sc.ctypes.data, fi.ctypes.data, status.ctypes.data)
        if st != OK:
            raise FisherBTError(st, lib().fbt_batch_last_error(self._h).decode())
        return ll, sc, fi.reshape(self.nf, 3, 3), status

    def set_exec(self, exec_: int):
        """WORKERS (0), GRAPH (1) or PERSISTENT (2) for the following calls."""
        st = lib().fbt_batch_set_exec(self._h, int(exec_))
        if st != OK:
            raise FisherBTError(st, "fbt_batch_set_exec: " +
                                lib().fbt_batch_last_error(self._h).decode())

    @property
    def exec(self) -> int:
        return int(lib().fbt_batch_get_exec(self._h))

    def fit(self, theta0=None, active=None, **opts):
        """Algorithm 1 for every field at once, one evaluation round per
        iteration of the fits (fbt_batch_fit).  theta0: (nf, 3) starts or
        None (L9); active: (nf,) flags or None (all).  Returns (list of result
        dicts, None for unselected fields; status (nf,); rounds)."""
        o, keep = _options(**opts)
        t0 = None
        if theta0 is not None:
            t0 = np.ascontiguousarray(theta0, dtype=np.float64).reshape(self.nf, 3)
        act = None
        if active is not None:
            act = np.ascontiguousarray(np.asarray(active, dtype=bool).astype(np.int32))
        res = (FitResult * max(1, self.nf))()
        status = np.zeros(self.nf, dtype=np.int32)
        rounds = _i32(0)
        st = lib().fbt_batch_fit(self._h, ctypes.byref(o), None if t0 is None else t0.ctypes.data,
                                 None if act is None else act.ctypes.data, res,
                                 status.ctypes.data, ctypes.byref(rounds))
        if st != OK:
            raise FisherBTError(st, lib().fbt_batch_last_error(self._h).decode())
        out = []
        for f in range(self.nf):
            if act is not None and not act[f]:
                out.append(None)
                continue
            d = _result(res[f])
            d["status"] = int(status[f])
            out.append(d)
        return out, status, int(rounds.value)

    def set_fit_threads(self, threads: int):
        """Fits of Batch.fit running at once (0: default)."""
        st = lib().fbt_batch_set_fit_threads(self._h, int(threads))
        if st != OK:
            raise FisherBTError(st, "fbt_batch_set_fit_threads(%d)" % threads)

    def set_tile(self, tile: int):
        """Tile rows of the persistent execution: 64, 128 or 0 (default)."""
        st = lib().fbt_batch_set_tile(self._h, int(tile))
        if st != OK:
            raise FisherBTError(st, "fbt_batch_set_tile(%d)" % tile)

    @property
    def tile(self) -> int:
        return int(lib().fbt_batch_get_tile(self._h))

    def round_stats(self):
        """(tasks, planner's makespan estimate in us, kernel ms) of the last
        persistent call."""
        nt, est, ms = _i64(0), ctypes.c_double(0), ctypes.c_double(0)
        st = lib().fbt_batch_round_stats(self._h, ctypes.byref(nt), ctypes.byref(est),
                                         ctypes.byref(ms))
        if st != OK:
            raise FisherBTError(st, "fbt_batch_round_stats")
        return int(nt.value), float(est.value), float(ms.value)

    def set_queues(self, queues: int):
        """Task queues of the persistent execution (1, 2, 4, 8; 0 default)."""
        st = lib().fbt_batch_set_queues(self._h, int(queues))
        if st != OK:
            raise FisherBTError(st, "fbt_batch_set_queues(%d)" % queues)

    def set_round_graph(self, on: bool = True):
        """Replay a HIP graph of the persistent round in later calls."""
        st = lib().fbt_batch_set_round_graph(self._h, int(bool(on)))
        if st != OK:
            raise FisherBTError(st, "fbt_batch_set_round_graph")

    def set_round_trace(self, on: bool = True):
        """Record a per-task trace in later persistent calls."""
        st = lib().fbt_batch_set_round_trace(self._h, int(bool(on)))
        if st != OK:
            raise FisherBTError(st, "fbt_batch_set_round_trace")

    def round_trace(self):
        """Trace of the last persistent call: (ntasks, 7) int64 array of
        (field, type, i, j, ticket time, ready time, end time) in wall-clock
        ticks, ticket order; None without a trace."""
        n = int(self.round_stats()[0])
        if n <= 0:
            return None
        raw = np.zeros(5 * n, dtype=np.int64)
        got = int(lib().fbt_batch_round_trace(self._h, raw.ctypes.data, n))
        if got <= 0:
            return None
        raw = raw.reshape(n, 5)
        ft, ij = raw[:, 0], raw[:, 1]
        return np.stack([ft >> 3, ft & 7, ij >> 16, ij & 0xFFFF, raw[:, 2], raw[:, 3], raw[:, 4]],
                        axis=1)

    def set_group_limit(self, npad: int, max_fields: int):
        st = lib().fbt_batch_set_group_limit(self._h, int(npad), int(max_fields))
        if st != OK:
            raise FisherBTError(st, "fbt_batch_set_group_limit")

    def group_limit(self, npad: int) -> int:
        return int(lib().fbt_batch_group_limit(self._h, int(npad)))

    def autotune(self, thetas, mode, path=None):
        """Time the candidate group limits per padded order and both
        executions on this workload; keep the fastest (written to `path` as
        JSON when given)."""
        th = np.ascontiguousarray(thetas, dtype=np.float64).reshape(self.nf, 3)
        md = np.ascontiguousarray(np.broadcast_to(np.asarray(mode, dtype=np.int32), (self.nf,)))
        st = lib().fbt_batch_autotune(self._h, th.ctypes.data, md.ctypes.data,
                                      None if path is None else str(path).encode())
        if st != OK:
            raise FisherBTError(st, lib().fbt_batch_last_error(self._h).decode())

    def load_tuning(self, path):
        st = lib().fbt_batch_load_tuning(self._h, str(path).encode())
        if st != OK:
            raise FisherBTError(st, "fbt_batch_load_tuning(%s)" % path)


def round_plan(n, mode, tile: int = 64, slots: int = 512, queues: int = 1):
    """Ticket order of the persistent execution's tasks (host only): an
    (ntasks, 4) int array of (field, type, i, j), the queue offsets (queue q
    holds rows qoff[q]:qoff[q+1]) and the planner's makespan estimate in
    microseconds."""
    n = np.ascontiguousarray(n, dtype=np.int64)
    md = np.ascontiguousarray(np.broadcast_to(np.asarray(mode, dtype=np.int32), n.shape))
    cnt, est = _i64(0), ctypes.c_double(0)
    st = lib().fbt_round_plan(n.size, n.ctypes.data, md.ctypes.data, int(tile), int(slots),
                              int(queues), ctypes.byref(cnt), None, None, ctypes.byref(est))
    if st != OK:
        raise FisherBTError(st, "fbt_round_plan")
    raw = np.zeros(2 * cnt.value, dtype=np.int32)
    qoff = np.zeros(int(queues) + 1, dtype=np.int64)
    st = lib().fbt_round_plan(n.size, n.ctypes.data, md.ctypes.data, int(tile), int(slots),
                              int(queues), ctypes.byref(cnt), raw.ctypes.data, qoff.ctypes.data,
                              None)
    if st != OK:
        raise FisherBTError(st, "fbt_round_plan")
    ft, ij = raw[0::2], raw[1::2]
    out = np.stack([ft >> 3, ft & 7, ij >> 16, ij & 0xFFFF], axis=1)
    return out, qoff, float(est.value)


def round_task_deps(T: int, mode: int, field: int, type_: int, i: int, j: int):
    """The persistent kernel's waits [(counter, value)] and advanced counters
    for one task of a field with T tiles (host only)."""
    off = np.zeros(4, dtype=np.int32)
    need = np.zeros(4, dtype=np.int32)
    pub = np.zeros(4, dtype=np.int32)
    npub = _i32(0)
    k = lib().fbt_round_task_deps(int(T), int(mode), (field << 3) | type_, (i << 16) | j,
                                  off.ctypes.data, need.ctypes.data, pub.ctypes.data,
                                  ctypes.byref(npub))
    return list(zip(off[:k].tolist(), need[:k].tolist())), pub[:npub.value].tolist()
