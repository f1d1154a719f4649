#!/usr/bin/env python3
"""Throughput of the exact Matern log-likelihood + score + Fisher evaluation
(Algorithm 3) on one MI355X.

One step = one evaluation of (l, grad l, I) over the full n x n covariance at
the workload's theta: covariance and derivative generation, tiled FP64
Cholesky, log-determinant and solve, the two triangular solves forming
W_i = L^{-1} Sigma_i L^{-T} and the trace reductions.  Inputs are resident on
the device before timing starts.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the seeded input generator lives beside the tests (shared by tests and bench)
sys.path.insert(0, os.path.join(ROOT, "tests"))

METRIC = "loglik+score+Fisher evals/s at n=20k, FP64 vs mixed; % of MFMA peak"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_MFMA_TFLOPS = 157.3   # dense FP32 matrix peak of MI355X
PEAK_BF16_MFMA_TFLOPS = 2500.0  # dense BF16 matrix peak of MI355X
# timing classes whose updates the mixed forms run in low precision (two-sided W phase)
LOWP_CLASSES = ("twosided_update", "twosided_lookahead", "deferred_update")
PEAK_HBM_GBS = 8000.0
# timing class -> kernel that implements it (for the counter summaries)
DOMINANT_KERNEL = {"left_update": "k_update_nn", "cholesky_update": "k_update_lower",
                   "right_update": "k_update_lower", "twosided_update": "k_syr2k_lower",
                   "deferred_update": "k_update_nn"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    """CPU model and the thread counts the oracle runs with (OpenMP for its
    C part, the BLAS behind numpy/SciPy for its LAPACK calls)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        import threadpoolctl

        blas = [{"api": i.get("internal_api"), "threads": i.get("num_threads")}
                for i in threadpoolctl.threadpool_info()]
    except Exception:  # threadpoolctl missing or failing: record nothing
        blas = None
    omp = os.environ.get("OMP_NUM_THREADS")
    return {"cpu": model, "logical_cpus": os.cpu_count(),
            "omp_threads": int(omp) if omp and omp.isdigit() else None, "blas": blas}


def cpu_baseline(n_full, n_sample, theta, seed):
    """The oracle as it stands, one evaluation on a bounded sample of the same
    workload (the same design and theta at a smaller n), scaled to the full n
    by n^3 (the evaluation is O(n^3))."""
    import oracle
    import synth

    oracle.build(force=False)
    locs, z, _ = synth.dataset(n_sample, theta, seed)
    t0 = time.perf_counter()
    oracle.evaluate(locs, z, theta)
    dt = time.perf_counter() - t0
    host = host_info()
    threads = host["omp_threads"] or host["logical_cpus"]
    return {"value": (1.0 / dt) * (n_sample / n_full) ** 3, "unit": "evals/s",
            "cores": threads, "kind": "oracle",
            "sample": "one oracle evaluation at n=%d (uniform locations, theta=%s) took %.2f s on "
                      "the host; scaled by (%d/%d)^3 to n=%d" % (n_sample, list(theta), dt, n_sample,
                                                              n_full, n_full),
            "sample_seconds": dt, "host": host}


def cpu_full(args):
    """One oracle evaluation at the full benchmark size (minutes of host
    time), with the host's CPU model and thread counts."""
    import oracle
    import synth

    w = dict(synth.WORKLOADS["n20k"])
    oracle.build(force=False)
    locs, z, _ = synth.dataset(args.n, w["theta_true"], w["seed"])
    log("oracle evaluation at n=%d ..." % args.n)
    t0 = time.perf_counter()
    r = oracle.evaluate(locs, z, w["theta_true"],
                        progress=lambda what: log("  %s (%.0f s)" % (what, time.perf_counter() - t0)))
    dt = time.perf_counter() - t0
    print(json.dumps({"what": "one oracle evaluation (Eqs. (1)-(3)) at n=%d, theta=%s"
                              % (args.n, list(w["theta_true"])),
                      "seconds": dt, "evals_per_s": 1.0 / dt, "loglik": r["loglik"],
                      "host": host_info()}), flush=True)


def kernel_source_sha256():
    """SHA-256 of the evaluation kernels' source: fbt_kernels.hip followed by
    fbt_device.h (the MFMA wrapper and the Matern entries it includes)."""
    import hashlib

    h = hashlib.sha256()
    for name in ("fbt_kernels.hip", "fbt_device.h"):
        with open(os.path.join(ROOT, "paper_2601_11437_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE passes, each scaled by what the
    same counter reads for a plain copy of known size).  None when no summary
    exists for this kernel or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "%s_n20k_pmc.md" % kernel)
    if not os.path.exists(path):
        return None, "no counter summary for this kernel"
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic_json:"):
                rec = json.loads(line.split(":", 1)[1])
    if rec is None:
        return None, "counter summary has no traffic_json line"
    if rec["source_sha256"] != kernel_source_sha256():
        return None, "kernel source changed since the counters were taken"
    b = 1024.0 * (rec["fetch_kib_per_dispatch"] * rec["fetch_scale"] +
                  rec["write_kib_per_dispatch"] * rec["write_scale"])
    return b, "rocprofv3 --pmc, %s" % os.path.relpath(path, ROOT)


def measured_gen_flops():
    """FP64 vector flops of one generation launch of Sigma, Sigma_alpha and
    Sigma_nu at the benchmark's n and theta, from the committed counter summary
    (rocprofv3 --pmc SQ_INSTS_VALU_{FMA,ADD,MUL}_F64: 64 (2 FMA + ADD + MUL)
    per launch).  None when there is none or the kernel source changed."""
    path = os.path.join(ROOT, "profiles", "k_gen_n20k_valu.md")
    if not os.path.exists(path):
        return None, "no counter summary for k_gen"
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("valu_json:"):
                rec = json.loads(line.split(":", 1)[1])
    if rec is None:
        return None, "counter summary has no valu_json line"
    if rec["source_sha256"] != kernel_source_sha256():
        return None, "kernel source changed since the counters were taken"
    return rec["fp64_valu_flops_per_launch"], "rocprofv3 --pmc, %s" % os.path.relpath(path, ROOT)


def copy_calibration():
    """A plain 1 GiB device-to-device copy, three times, for scaling the HBM
    byte counters (run under rocprofv3 --pmc)."""
    import torch

    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8,
                      "repeats": 3}), flush=True)


def round_trace_summary(tr, bt, kernel_ms):
    """Per-task-type breakdown of a persistent round's trace: workgroup time
    busy and waiting, task counts, the products' executed FP64 rate per
    workgroup, and the share of busy workgroup time per type."""
    import numpy as np

    f, ty, i, j, t_take, t_ready, t_end = tr.T
    tick_ms = 1e-5  # the device wall clock runs at 100 MHz
    busy = (t_end - t_ready) * tick_ms
    wait = (t_ready - t_take) * tick_ms
    fl = np.zeros(len(ty))
    b3 = 2.0 * bt ** 3
    m = ty == 1
    fl[m] = 2.0 * bt * bt * (j[m] * bt) + np.where(i[m] > j[m], b3, 0.0)
    m = ty == 2
    fl[m] = 2.0 * bt * bt * (i[m] * bt) + b3
    m = ty == 3
    fl[m] = 2.0 * (2.0 * bt * bt * (j[m] * bt) + b3)
    span_ms = (t_end.max() - t_take.min()) * tick_ms
    out = {"kernel_ms": kernel_ms, "trace_span_ms": span_ms,
           "workgroup_busy_ms": float(busy.sum()), "workgroup_wait_ms": float(wait.sum()),
           "executed_flops": float(fl.sum()), "types": {}}
    for k, name in enumerate(("generation", "cholesky", "forward_subst", "w_tiles", "reduce")):
        m = ty == k
        bsum = float(busy[m].sum())
        out["types"][name] = {
            "tasks": int(m.sum()), "busy_ms": bsum, "wait_ms": float(wait[m].sum()),
            "busy_share": bsum / float(busy.sum()),
            "mean_busy_us": 1e3 * bsum / max(1, int(m.sum())),
            "tflops_per_workgroup": (float(fl[m].sum()) / (bsum * 1e-3) / 1e12) if fl[m].sum() else None}
    return out


def batch_bench(args):
    """One Fisher-BT round over many independent fields (loglik + score +
    Fisher for every field), through the batch executor."""
    import numpy as np

    import paper_2601_11437_amd as fbt
    import synth

    t0 = time.perf_counter()
    fields, thetas = synth.batch_workload(args.batch)
    log("batch data: %d fields generated in %.1f s" % (len(fields), time.perf_counter() - t0))
    b = fbt.Batch(args.batch_workers)
    b.set_fields(fields)
    gen = synth.rng(5000 + 104729)
    redraws = 0
    for _ in range(50):   # evaluation points whose covariance is not PD are redrawn
        _, _, _, st = b.eval(thetas, fbt.Batch.LOGLIK)
        bad = st != fbt.OK
        if not bad.any():
            break
        redraws += int(bad.sum())
        thetas = synth.batch_redraw_thetas(thetas, bad, gen)
    def timed():
        for _ in range(args.warmup):
            b.eval(thetas, fbt.Batch.EVAL)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = b.eval(thetas, fbt.Batch.EVAL)
        return time.perf_counter() - t0, r

    # the worker execution without group limits, for comparison
    dt_workers, _ = timed()
    log("workers, no limits: %.1f ms per round" % (1e3 * dt_workers / args.steps))
    tune = None
    if args.batch_exec == "graph":
        b.set_exec(fbt.Batch.GRAPH)
    elif args.batch_exec == "persistent":
        b.set_exec(fbt.Batch.PERSISTENT)
        if args.batch_tile:
            b.set_tile(args.batch_tile)
    elif args.batch_exec == "tuned":
        t0 = time.perf_counter()
        path = os.path.join(tempfile.gettempdir(), "fisherbt_batch_tuning.json")
        b.autotune(thetas, fbt.Batch.EVAL, path)
        with open(path) as f:
            tune = json.load(f)
        tune["tuning_seconds"] = time.perf_counter() - t0
        log("autotune: %.1f s, exec %s, tile %s, limits %s"
            % (tune["tuning_seconds"], ("workers", "graph", "persistent")[tune["exec"]],
               tune.get("tile"), tune["limits"]))
    dt, (ll, sc, fi, st) = timed()
    b_exec = b.exec
    persistent = b_exec == fbt.Batch.PERSISTENT
    round_info = None
    if persistent:
        ntasks, plan_us, kernel_ms = b.round_stats()
        round_info = {"tile": b.tile, "tasks": ntasks, "planner_estimate_ms": plan_us / 1e3,
                      "kernel_ms_last_round": kernel_ms,
                      "launches_per_round": 1}
        log("persistent round: tile %d, %d tasks, kernel %.1f ms" % (b.tile, ntasks, kernel_ms))
        if args.round_trace:
            # one more round with the per-task trace on (outside the timed rounds)
            b.set_round_trace(True)
            b.eval(thetas, fbt.Batch.EVAL)
            round_info["trace"] = round_trace_summary(b.round_trace(), b.tile,
                                                      b.round_stats()[2])
            b.set_round_trace(False)
    b.close()
    ns = np.array([z.size for _, z in fields], dtype=np.float64)
    # n^3 / 3 (factorisation) + 2 n^3 (two-sided W phase of both derivative
    # matrices) per field: the algorithmic count, which the two-sided form
    # executes (plus the diagonal blocks' zero padding)
    exec_flops = float(np.sum(7.0 * ns ** 3 / 3.0)) * args.steps
    nf = len(fields)
    out = {"metric": "loglik+score+Fisher field evaluations/s, %d fields n~U[500,4000]" % nf,
           "value": nf * args.steps / dt, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "%d independent Matern fields, n_f ~ U[500, 4000] uniform points, "
                                  "theta_f uniform in [0.5,2]x[0.02,0.3]x[0.3,2.5], one full "
                                  "evaluation per field per step" % nf,
                      "workers": args.batch_workers, "theta_redraws": redraws,
                      "exec": args.batch_exec,
                      "exec_used": ("workers", "graph", "persistent")[b_exec]},
           "tuning": tune,
           "persistent_round": round_info,
           "ms_per_step_workers_untuned": 1e3 * dt_workers / args.steps,
           "algorithmic_flops_per_round": exec_flops / args.steps,
           "executed_tflops": exec_flops / dt / 1e12,
           "fp64_frac": exec_flops / dt / 1e12 / PEAK_FP64_TFLOPS,
           "failed_fields": int(np.sum(st != fbt.OK))}
    print(json.dumps(out), flush=True)


def batch_fit_bench(args):
    """Fisher-BT for many replicate fields at once (fbt_batch_fit): every
    field's fit from the L9 start, all fits' evaluations of one iteration in
    one round (one persistent launch)."""
    import numpy as np

    import paper_2601_11437_amd as fbt
    import synth

    t0 = time.perf_counter()
    approx = []
    fields, theta_true = synth.batch_fit_workload(
        args.batch_fit, approx=approx, draw="rff",
        progress=lambda f: (f + 1) % 32 == 0 and log("batch-fit data: %d fields" % (f + 1)))
    log("batch-fit data: %d fields generated in %.1f s (%d by the approximate draw)"
        % (len(fields), time.perf_counter() - t0, len(approx)))
    b = fbt.Batch(args.batch_workers)
    b.set_fields(fields)
    b.set_exec(fbt.Batch.PERSISTENT)
    if args.batch_tile:
        b.set_tile(args.batch_tile)
    # one untimed round builds the plan and the device arena
    b.eval(theta_true, fbt.Batch.EVAL)
    t0 = time.perf_counter()
    fits, st, rounds = b.fit()
    dt = time.perf_counter() - t0
    b.close()
    nf = len(fields)
    ok = [f for f in fits if f is not None and f["status"] == fbt.OK]
    conv = sum(1 for f in ok if f["converged"] and not f["used_nelder_mead"])
    nm = sum(1 for f in ok if f["used_nelder_mead"])
    ns = np.array([z.size for _, z in fields], dtype=np.float64)
    th = np.array([f["theta"] for f in fits])
    out = {"metric": "Fisher-BT fits of %d replicate fields, n~U[500,4000]: wall time" % nf,
           "value": dt, "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "%d fields, n_f ~ U[500, 4000] uniform points, true theta_f "
                                  "uniform in [0.5,2]x[0.02,0.3]x[0.3,2.5], one realisation "
                                  "each (random-Fourier-feature draw, 4096 features); "
                                  "Algorithm 1 from the L9 start" % nf,
                      "exec": "persistent", "tile": args.batch_tile or 128},
           "fields_approximate_draw": len(approx),
           "rounds": rounds, "ms_per_round": 1e3 * dt / max(1, rounds),
           "fits_ok": len(ok), "converged_by_scoring": conv, "nelder_mead": nm,
           "loglik_calls_total": int(sum(f["n_loglik_calls"] for f in ok)),
           "grad_calls_total": int(sum(f["n_grad_calls"] for f in ok)),
           "median_rel_err_vs_true": float(np.median(np.abs(th - theta_true) / theta_true)),
           "sum_n_cubed": float(np.sum(ns ** 3))}
    print(json.dumps(out), flush=True)


def fit_bench(args):
    """Algorithm 1 end to end at the benchmark size: Fisher-BT from the L9
    start within the paper's simulation bounds, in FP64 and in the mixed form;
    wall time per fit, call counts and the mixed form's theta-hat error."""
    import numpy as np

    import paper_2601_11437_amd as fbt
    import synth

    w = dict(synth.WORKLOADS["n20k"])
    n = args.n
    locs, z, _ = synth.dataset(n, w["theta_true"], w["seed"])
    ctx = fbt.Context(0)
    ctx.set_data(locs, z)
    lo, hi = (0.01, 0.01, 0.01), (5.0, 5.0, 2.0)
    ctx.loglik(w["theta_true"])   # warm-up
    fits = {}
    for name, prec in (("fp64", fbt.FP64), ("mixed", fbt.MIXED_FP32)):
        ctx.set_precision(prec)
        t0 = time.perf_counter()
        r = ctx.fit(lo=lo, hi=hi)
        dt = time.perf_counter() - t0
        fits[name] = {"seconds": dt, "theta": r["theta"].tolist(), "loglik": r["loglik"],
                      "n_loglik_calls": r["n_loglik_calls"], "n_grad_calls": r["n_grad_calls"],
                      "n_iter": r["n_iter"], "used_nelder_mead": bool(r["used_nelder_mead"]),
                      "n_fp64_evals": r["n_fp64_evals"], "precision_switch": r["precision_switch"],
                      "converged": bool(r["converged"]), "grad_norm": float(np.linalg.norm(r["score"]))}
        log("%s fit: %.2f s, theta %s" % (name, dt, np.round(r["theta"], 6)))
    ctx.close()
    t64, tm = np.array(fits["fp64"]["theta"]), np.array(fits["mixed"]["theta"])
    out = {"metric": "Fisher-BT fit wall time at n=%d (L9 start, paper bounds)" % n,
           "value": fits["fp64"]["seconds"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": 1e3 * fits["fp64"]["seconds"], "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "Matern GRF, n=%d uniform on [0,1]^2, theta_true=%s; one full "
                                  "Fisher-BT fit" % (n, list(w["theta_true"]))},
           "fits": fits,
           "mixed_theta_rel_err_vs_fp64": (np.abs(tm - t64) / np.abs(t64)).tolist()}
    print(json.dumps(out), flush=True)


def grid_bench(args):
    """The 3 x 3 simulation grid at n = 10,000 (100 x 100 jittered grid):
    one FP64 Fisher-BT fit (L9 start, paper bounds) per true theta."""
    import numpy as np

    import paper_2601_11437_amd as fbt
    import synth

    ctx = fbt.Context(0)
    fits, total = [], 0.0
    for ib in range(3):
        for inu in range(3):
            w = synth.grid_workload(ib, inu)
            t0 = time.perf_counter()
            locs, z, info = synth.dataset(w["n"], w["theta_true"], w["seed"], design=w["design"])
            tg = time.perf_counter() - t0
            ctx.set_data(locs, z)
            t0 = time.perf_counter()
            r = ctx.fit()
            dt = time.perf_counter() - t0
            total += dt
            fits.append({"theta_true": list(w["theta_true"]), "seed": w["seed"],
                         "redraws": info["redraws"], "seconds": dt, "theta_hat": r["theta"].tolist(),
                         "loglik": r["loglik"], "grad_norm": float(np.linalg.norm(r["score"])),
                         "n_loglik_calls": r["n_loglik_calls"], "n_grad_calls": r["n_grad_calls"],
                         "n_iter": r["n_iter"], "used_nelder_mead": r["used_nelder_mead"],
                         "converged": r["converged"]})
            log("grid theta_true %s: data %.1f s, fit %.2f s, theta_hat %s, %d l / %d grad calls%s"
                % (w["theta_true"], tg, dt, np.round(r["theta"], 5), r["n_loglik_calls"],
                   r["n_grad_calls"], ", Nelder-Mead" if r["used_nelder_mead"] else ""))
    ctx.close()
    out = {"metric": "Fisher-BT fits/s, 3x3 grid at n=10,000 (jittered 100x100 grid)",
           "value": len(fits) / total, "unit": "fits/s", "n_gpus": 1, "steps": len(fits),
           "warmup": 0, "ms_per_step": 1e3 * total / len(fits), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "100x100 grid on [0,1]^2 with +-0.4 cell jitter; sigma2 = 1, "
                                  "beta in {0.03, 0.1, 0.3}, nu in {0.5, 1.0, 2.5}; one "
                                  "realisation and one FP64 Fisher-BT fit per setting"},
           "fits": fits}
    print(json.dumps(out), flush=True)


def precision_bench(args):
    """FP64 against the mixed forms at n = 50,000 (theta = (1, 0.05, 0.8)):
    one evaluation each, errors of l, score and Fisher against FP64."""
    import numpy as np

    import paper_2601_11437_amd as fbt
    import synth

    w = synth.WORKLOADS["n50k"]
    n, theta = args.precision_n or w["n"], w["theta_true"]
    gen = synth.rng(w["seed"])
    locs = synth.uniform_locations(n, gen)
    z = synth.rff_field(locs, theta, gen)
    ctx = fbt.Context(0)
    ctx.set_data(locs, z)
    res = {}
    # the _ALL forms as they are by default, and with two refinement steps of w
    for name, prec, refine in (("fp64", fbt.FP64, 0), ("mixed_fp32", fbt.MIXED_FP32, 0),
                               ("mixed_fp32_all", fbt.MIXED_FP32_ALL, 0),
                               ("mixed_fp32_all_refined", fbt.MIXED_FP32_ALL, 2),
                               ("mixed_bf16", fbt.MIXED_BF16, 0),
                               ("mixed_bf16_all", fbt.MIXED_BF16_ALL, 0),
                               ("mixed_bf16_all_refined", fbt.MIXED_BF16_ALL, 2)):
        ctx.set_precision(prec)
        ctx.set_refinement(refine)
        try:
            ctx.loglik(theta)                    # untimed (buffers, FP32 copies)
            t0 = time.perf_counter()
            ll_only = ctx.loglik(theta)
            t1 = time.perf_counter()
            terms = ctx.eval_terms(theta)        # reuses the factor of the loglik call
            t2 = time.perf_counter()
            ll, sc, fi = ctx.eval(theta)          # factors afresh
            t3 = time.perf_counter()
        except fbt.FisherBTError as e:
            res[name] = {"status": str(e)}
            log("%s: %s" % (name, e))
            continue
        res[name] = {"loglik": ll, "score": sc.tolist(), "fisher": fi.tolist(), "terms": terms.tolist(),
                     "loglik_s": t1 - t0, "eval_s": t3 - t2, "w_phase_s": t2 - t1}
        log("%s: loglik %.3f s, eval %.3f s" % (name, t1 - t0, t3 - t2))
    ctx.set_refinement(0)
    if args.precision_fits:
        # Fisher-BT from the L9 start in FP64 and in the FP32 and BF16 mixed forms
        # (both switch to FP64 near the optimum).  No Nelder-Mead fallback: a
        # fit that exhausts its derivative budget reports so (the fallback's
        # hundreds of log-likelihood calls would take minutes at this size).
        lo, hi = (0.01, 0.01, 0.01), (5.0, 5.0, 2.0)
        for name, prec in (("fp64", fbt.FP64), ("mixed_fp32", fbt.MIXED_FP32),
                           ("mixed_bf16", fbt.MIXED_BF16)):
            ctx.set_precision(prec)
            t0 = time.perf_counter()
            r = ctx.fit(lo=lo, hi=hi, nelder_mead=0, callback=lambda it, th, ll, g, fi: log(
                "  %s fit iterate %d: theta %s, |grad| %.3g" % (name, it, np.round(th, 6),
                                                               np.linalg.norm(g))))
            dt = time.perf_counter() - t0
            res[name]["fit"] = {"seconds": dt, "theta": r["theta"].tolist(), "loglik": r["loglik"],
                                "status": int(r["status"]),
                                "n_loglik_calls": r["n_loglik_calls"],
                                "n_grad_calls": r["n_grad_calls"], "converged": r["converged"],
                                "used_nelder_mead": r["used_nelder_mead"],
                                "precision_switch": r["precision_switch"],
                                "grad_norm": float(np.linalg.norm(r["score"]))}
            log("%s fit: %.1f s, theta %s" % (name, dt, np.round(r["theta"], 7)))
        ctx.set_precision(fbt.FP64)
        t64 = np.array(res["fp64"]["fit"]["theta"])
        for name in ("mixed_fp32", "mixed_bf16"):
            tm = np.array(res[name]["fit"]["theta"])
            res[name]["fit"]["theta_rel_err_vs_fp64"] = (np.abs(tm - t64) / np.abs(t64)).tolist()
    ctx.close()
    ref = res["fp64"]
    t = np.array(ref["terms"])
    scale = np.array([(t[1] + n) / (2 * theta[0]), 0.5 * (abs(t[2]) + abs(t[4])),
                      0.5 * (abs(t[3]) + abs(t[5]))])
    fd = np.diag(np.array(ref["fisher"]))
    for name in ("mixed_fp32", "mixed_fp32_all", "mixed_fp32_all_refined", "mixed_bf16",
                 "mixed_bf16_all", "mixed_bf16_all_refined"):
        r = res[name]
        if "loglik" not in r:
            continue
        r["loglik_rel_err_vs_fp64"] = abs(r["loglik"] - ref["loglik"]) / abs(ref["loglik"])
        r["loglik_speedup_vs_fp64"] = ref["loglik_s"] / r["loglik_s"]
        r["score_err_per_term_vs_fp64"] = (np.abs(np.array(r["score"]) - ref["score"]) / scale).tolist()
        r["fisher_rel_err_vs_fp64"] = float(np.max(np.abs(np.array(r["fisher"]) - ref["fisher"])
                                                   / np.sqrt(np.outer(fd, fd))))
        r["eval_speedup_vs_fp64"] = ref["eval_s"] / r["eval_s"]
    out = {"metric": "loglik+score+Fisher evals/s at n=%d, FP64 vs mixed" % n,
           "value": 1.0 / ref["eval_s"], "unit": "evals/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": 1e3 * ref["eval_s"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "n=%d uniform on [0,1]^2, theta=%s; data by %d random Fourier "
                                  "features of the Matern field" % (n, list(theta), 4096)},
           "forms": res}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--cpu-sample-n", type=int, default=10000,
                    help="n of the oracle's timed sample (the CPU baseline)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only time one oracle evaluation at the full n on the host")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision and adjoint comparisons (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB copy used to scale the HBM byte counters")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead of the n=20k evaluation, time one round over this many fields")
    ap.add_argument("--batch-workers", type=int, default=2)
    ap.add_argument("--batch-fit", type=int, default=0,
                    help="Fisher-BT fits of this many replicate fields at once "
                         "(persistent execution, one round per iteration)")
    ap.add_argument("--round-trace", action="store_true",
                    help="persistent execution: one extra traced round, its per-task-type "
                         "breakdown in the JSON line")
    ap.add_argument("--batch-tile", type=int, default=0,
                    help="tile rows of the persistent execution (64, 128; 0: default)")
    ap.add_argument("--batch-exec", choices=("workers", "graph", "tuned", "persistent"),
                    default="tuned",
                    help="batch execution: worker threads, one HIP graph per round, the "
                         "autotuner's choice of execution, tile and group limits, or one "
                         "persistent launch per round")
    ap.add_argument("--fit", action="store_true",
                    help="instead of the evaluation rate, time one full Fisher-BT fit (FP64 and mixed)")
    ap.add_argument("--grid", action="store_true",
                    help="instead of the evaluation rate, the 3x3 grid of FP64 fits at n=10,000")
    ap.add_argument("--precision", action="store_true",
                    help="instead of the evaluation rate, FP64 vs the mixed forms at n=50,000")
    ap.add_argument("--precision-n", type=int, default=0,
                    help="with --precision, the number of points (default 50,000)")
    ap.add_argument("--precision-fits", action="store_true",
                    help="with --precision, also one FP64 and two mixed Fisher-BT fits (minutes)")
    args = ap.parse_args()
    if args.grid and args.gpus == 1:
        grid_bench(args)
        return
    if args.precision and args.gpus == 1:
        precision_bench(args)
        return
    if args.fit and args.gpus == 1:
        fit_bench(args)
        return
    if args.batch_fit and args.gpus == 1:
        batch_fit_bench(args)
        return
    if args.batch and args.gpus == 1:
        batch_bench(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.cpu_full:
        cpu_full(args)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library does not shard the single-field "
              "evaluation across GPUs (see the design notes); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import paper_2601_11437_amd as fbt
    import synth

    w = dict(synth.WORKLOADS["n20k"])
    n = args.n
    theta = w["theta_true"]
    t0 = time.perf_counter()
    locs, z, info = synth.dataset(n, theta, w["seed"])
    log("data: n=%d generated in %.1f s" % (n, time.perf_counter() - t0))

    ctx = fbt.Context(0)
    ctx.set_data(locs, z)
    for i in range(args.warmup):
        ctx.eval(theta)
        log("warmup step %d done" % i)
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        ll, score, fisher = ctx.eval(theta)
        log("step %d done (loglik %.6f)" % (i, ll))
    dt = time.perf_counter() - t0
    tim = ctx.timing()
    ctx.set_timing(False)
    # loglik-only rate (Algorithm 2): generation of Sigma and the Cholesky phase
    t1 = time.perf_counter()
    for i in range(max(1, args.steps)):
        ctx.loglik(theta)
    dt_ll = (time.perf_counter() - t1) / max(1, args.steps)
    # the W phase alone: a derivative evaluation right after a log-likelihood
    # call at the same theta reuses its factor (generation of the derivative
    # matrices, the W phase and the trace reductions)
    dt_w = 0.0
    for i in range(max(1, args.steps)):
        ctx.loglik(theta)
        t1 = time.perf_counter()
        ctx.eval_terms(theta)
        dt_w += time.perf_counter() - t1
    dt_w /= max(1, args.steps)

    mixed = mixed_bf16 = adjoint = None
    if not args.no_mixed:
        tscale = ctx.eval_terms(theta)
        sscale = np.array([(tscale[1] + n) / (2 * theta[0]),
                           0.5 * (abs(tscale[2]) + abs(tscale[4])),
                           0.5 * (abs(tscale[3]) + abs(tscale[5]))])
        dd = np.sqrt(np.outer(np.diag(fisher), np.diag(fisher)))

        def mixed_form(prec, what):
            # a mixed form, same workload and steps, with its errors against FP64
            ctx.set_precision(prec)
            for i in range(args.warmup):
                ctx.eval(theta)
            t2 = time.perf_counter()
            for i in range(args.steps):
                llm, scm, fim = ctx.eval(theta)
            dt_mix = time.perf_counter() - t2
            ctx.set_precision(fbt.FP64)
            return {"precision": what, "value": args.steps / dt_mix, "unit": "evals/s",
                    "ms_per_step": 1e3 * dt_mix / args.steps, "speedup_vs_fp64": dt / dt_mix,
                    "loglik_rel_err_vs_fp64": abs(llm - ll) / abs(ll),
                    "score_err_per_term_vs_fp64": (np.abs(scm - score) / sscale).tolist(),
                    "fisher_rel_err_vs_fp64": float(np.max(np.abs(fim - fisher) / dd))}

        mixed = mixed_form(fbt.MIXED_FP32,
                           "trace-phase updates FP32 MFMA (FP32 accumulation); factorisation, log-det, "
                           "solves of the diagonal blocks, Bessel terms and reductions FP64")
        log("mixed: %.1f ms per step" % mixed["ms_per_step"])
        mixed_bf16 = mixed_form(fbt.MIXED_BF16,
                                "trace-phase updates with bfloat16 operands on MFMA (FP32 sums per "
                                "256-deep slice); the rest as in the FP32 form; not a fitting form")
        log("mixed bf16: %.1f ms per step" % mixed_bf16["ms_per_step"])
        # adjoint gradient (log-likelihood + score, no Fisher), FP64
        ctx.grad(theta)
        t3 = time.perf_counter()
        for i in range(args.steps):
            lla, sca = ctx.grad(theta)
        dt_adj = time.perf_counter() - t3
        adjoint = {"what": "loglik + score by the adjoint form (no Fisher information), FP64",
                   "value": args.steps / dt_adj, "unit": "grads/s",
                   "ms_per_step": 1e3 * dt_adj / args.steps,
                   "score_err_per_term_vs_eval": (np.abs(sca - score) / sscale).tolist(),
                   "loglik_equal": bool(lla == ll)}
        log("adjoint: %.1f ms per gradient" % (1e3 * dt_adj / args.steps))

    evals_per_s = args.steps / dt
    phases = {}
    for name, v in tim.items():
        if v["launches"]:
            phases[name] = {"launches_per_step": v["launches"] / args.steps,
                            "ms_per_step": v["ms"] / args.steps,
                            "tflops": (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["flops"] and v["ms"] else None}
    # dominant kernel: the one with the most time
    dom = max((k for k in tim if tim[k]["flops"] > 0), key=lambda k: tim[k]["ms"])
    d = tim[dom]
    achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
    traffic, traffic_src = measured_traffic(DOMINANT_KERNEL.get(dom, dom))
    # the counted L2-miss bytes over the launch time: the kernel's rate against
    # the HBM peak (an upper bound on its HBM traffic; the Infinity Cache serves
    # part of the misses)
    traffic_gbs = traffic / (d["ms"] / d["launches"] * 1e-3) / 1e9 if traffic else None
    roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                "traffic_unit": "bytes per launch", "traffic_source": traffic_src,
                "traffic_GBps": traffic_gbs,
                "traffic_frac_hbm_peak": traffic_gbs / PEAK_HBM_GBS if traffic_gbs else None,
                "launches": d["launches"], "avg_launch_ms": d["ms"] / d["launches"],
                "flops_per_launch": d["flops"] / d["launches"]}
    total_fl = sum(v["flops"] for v in tim.values())
    total_ms = sum(v["ms"] for v in tim.values())
    # fractions of the FP64 peak per phase: algorithmic flops (n^3 / 3 for the
    # Cholesky phase, 2 n^3 for the W phase of both derivative matrices,
    # 7 n^3 / 3 for the evaluation) and the flops the kernels execute
    ms_step = 1e3 * dt / args.steps
    two_sided = tim.get("twosided_update", {}).get("launches", 0) > 0
    w_exec = 2.0 * n ** 3 if two_sided else 8.0 * n ** 3 / 3.0

    def frac(fl, ms):
        return {"tflops": fl / (ms * 1e-3) / 1e12, "frac_fp64_peak": fl / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}

    phase_fracs = {
        "whole_eval": dict(ms=ms_step, algorithmic_flops=7.0 * n ** 3 / 3.0,
                           executed_flops=n ** 3 / 3.0 + w_exec,
                           algorithmic=frac(7.0 * n ** 3 / 3.0, ms_step),
                           executed=frac(n ** 3 / 3.0 + w_exec, ms_step)),
        "cholesky_phase": dict(ms=1e3 * dt_ll, algorithmic_flops=n ** 3 / 3.0,
                               note="fbt_loglik: generation of Sigma, factorisation, log det, "
                                    "forward solve", algorithmic=frac(n ** 3 / 3.0, 1e3 * dt_ll)),
        "w_phase": dict(ms=1e3 * dt_w, algorithmic_flops=2.0 * n ** 3, executed_flops=w_exec,
                        form="two-sided reduction" if two_sided else "block solves",
                        note="derivative evaluation on the log-likelihood call's factor: "
                             "generation of Sigma_alpha and Sigma_nu, W phase, trace reductions",
                        algorithmic=frac(2.0 * n ** 3, 1e3 * dt_w), executed=frac(w_exec, 1e3 * dt_w)),
    }
    def mixed_roofline(form, peak_lowp):
        # lower bound on a mixed evaluation's time with every flop at its unit's
        # peak: the W phase's low-precision updates at the low-precision MFMA
        # peak, the rest at the FP64 peak (flops per class from the FP64 run's
        # timing classes: the schedule is the same)
        if form is None or not two_sided:
            return None
        lowp = sum(tim[k]["flops"] for k in LOWP_CLASSES if k in tim) / args.steps
        f64 = total_fl / args.steps - lowp
        bound_ms = 1e3 * (f64 / (PEAK_FP64_TFLOPS * 1e12) + lowp / (peak_lowp * 1e12))
        return {"fp64_flops": f64, "lowp_flops": lowp, "peak_fp64": PEAK_FP64_TFLOPS,
                "peak_lowp": peak_lowp, "unit": "TFLOP/s", "bound_ms": bound_ms,
                "frac": bound_ms / form["ms_per_step"]}

    # the generation (k_gen, all three matrices) is bound by FP64 vector
    # arithmetic (the quadrature of K_nu), not by MFMA or HBM: its counted FP64
    # vector flops over its launch time measured here, against the FP64 vector
    # peak (256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s)
    gen_fl, gen_src = measured_gen_flops()
    if "generation" in phases and gen_fl:
        g = tim["generation"]
        ach = gen_fl / (g["ms"] / g["launches"] * 1e-3) / 1e12
        phases["generation"]["roofline"] = {"bound": "alu", "achieved": ach,
                                            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                            "frac": ach / PEAK_FP64_TFLOPS,
                                            "flops_per_launch": gen_fl, "source": gen_src}
    if mixed is not None:
        mixed["roofline"] = mixed_roofline(mixed, PEAK_FP32_MFMA_TFLOPS)
    if mixed_bf16 is not None:
        mixed_bf16["roofline"] = mixed_roofline(mixed_bf16, PEAK_BF16_MFMA_TFLOPS)
    out = {
        "metric": METRIC,
        "value": evals_per_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Matern GRF, n=%d uniform on [0,1]^2, theta=(sigma2, alpha, nu)=%s, "
                               "one loglik+score+Fisher evaluation per step" % (n, list(theta)),
                   "n": n, "theta": list(theta), "precision": "fp64", "tile": 256},
        "roofline": roofline,
        "whole_eval_tflops": total_fl / (total_ms * 1e-3) / 1e12 if total_ms else None,
        "fp64_frac_whole_eval": total_fl / dt / 1e12 / PEAK_FP64_TFLOPS,
        "phase_fractions": phase_fracs,
        "loglik_only_evals_per_s": 1.0 / dt_ll,
        "phases": phases,
        "mixed": mixed,
        "mixed_bf16": mixed_bf16,
        "adjoint_grad": adjoint,
        "result": {"loglik": ll, "score": score.tolist(), "fisher_diag": np.diag(fisher).tolist()},
    }
    ctx.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) at n=%d ..." % args.cpu_sample_n)
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_sample_n, theta, w["seed"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
