"""Writes the oracle's evaluations that the full-size GPU parity tests compare
against (Eqs. (1)-(3): log-likelihood, score, Fisher information and the
intermediate traces and quadratic forms):

  eval_n20k_oracle.json    the 20,000-point benchmark field at theta = (1, 0.1, 0.5)
                           (the benchmark's evaluation point) and at the oracle
                           fit's theta-hat (fit_n20k_oracle.json);
  eval_n10k_oracle.json    the 10,000-point differentiation field (theta_true =
                           (1, 0.1, 1.5)) at 20 parameter vectors drawn uniformly
                           from sigma2 in [0.5, 2], alpha in [0.02, 0.3], nu in
                           [0.3, 3] (seed 3001); a draw whose Sigma fails the
                           oracle's Cholesky is replaced by the next draw.  Each
                           point also records LAPACK's 1-norm condition estimate
                           of Sigma (dpocon on the oracle's factor).

It calls only the oracle and the seeded input generator.  The 20,000-point
evaluations take several minutes of host time each.

    python tests/golden/make_eval_goldens.py [n20k] [n10k]
"""
import json
import os
import platform
import sys
import time

import numpy as np
import scipy.linalg
import scipy.linalg.lapack as lapack

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import synth  # noqa: E402


def _record(r, theta, seconds):
    return {
        "theta": [float(t) for t in theta],
        "loglik": r["loglik"],
        "score": np.asarray(r["score"]).tolist(),
        "fisher": np.asarray(r["fisher"]).tolist(),
        "logdet": r["logdet"],
        "quad": r["quad"],
        "trace": r["trace"],
        "wSw": r["wSw"],
        "trAB_frobenius": r["trAB_frobenius"],
        "trAB_direct": r["trAB_direct"],
        "host_seconds": seconds,
    }


def _host():
    model = platform.processor()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu": model, "cpus": os.cpu_count()}


def n20k():
    w = dict(synth.WORKLOADS["n20k"])
    locs, z, info = synth.dataset(w["n"], w["theta_true"], w["seed"])
    with open(os.path.join(HERE, "fit_n20k_oracle.json")) as f:
        theta_hat = json.load(f)["theta"]
    points = []
    for theta in (w["theta_true"], theta_hat):
        t0 = time.perf_counter()
        r = oracle.evaluate(locs, z, theta)
        dt = time.perf_counter() - t0
        print("n20k theta=%s loglik=%r  (%.0f s)" % (list(theta), r["loglik"], dt), flush=True)
        points.append(_record(r, theta, dt))
    rec = {
        "what": "oracle log-likelihood, score and Fisher information (Eqs. (1)-(3)) on the "
                "20,000-point benchmark field",
        "workload": {"n": w["n"], "theta_true": list(w["theta_true"]), "seed": w["seed"],
                     "design": w["design"], "redraws": int(info["redraws"])},
        "points": points,
        "host": _host(),
    }
    out = os.path.join(HERE, "eval_n20k_oracle.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", out, flush=True)


def _cond1(locs, theta):
    """LAPACK's 1-norm condition estimate of Sigma(theta) (dpocon), or None if
    the Cholesky factorisation fails."""
    (S,) = oracle.cov_matrices(locs, theta, which=("S",))
    anorm = float(np.max(np.sum(np.abs(S), axis=0)))
    try:
        c = scipy.linalg.cholesky(S, lower=True, overwrite_a=True, check_finite=False)
    except np.linalg.LinAlgError:
        return None
    rcond, info = lapack.dpocon(c, anorm, uplo="L")
    return float(1.0 / rcond) if info == 0 and rcond > 0 else float("inf")


def n10k():
    w = dict(synth.WORKLOADS["n10k_diff"])
    locs, z, info = synth.dataset(w["n"], w["theta_true"], w["seed"])
    gen = synth.rng(3001)
    points, redraws = [], 0
    while len(points) < 20:
        theta = (gen.uniform(0.5, 2.0), gen.uniform(0.02, 0.3), gen.uniform(0.3, 3.0))
        kappa = _cond1(locs, theta)
        if kappa is None:
            redraws += 1
            print("n10k theta=%s not positive definite: redrawn" % (list(theta),), flush=True)
            continue
        t0 = time.perf_counter()
        r = oracle.evaluate(locs, z, theta)
        dt = time.perf_counter() - t0
        rec = _record(r, theta, dt)
        rec["cond1"] = kappa
        points.append(rec)
        print("n10k %d theta=%s cond1=%.2e loglik=%r (%.0f s)"
              % (len(points), list(np.round(theta, 6)), kappa, r["loglik"], dt), flush=True)
    rec = {
        "what": "oracle log-likelihood, score and Fisher information (Eqs. (1)-(3)) on the "
                "10,000-point differentiation field at 20 random parameter vectors",
        "workload": {"n": w["n"], "theta_true": list(w["theta_true"]), "seed": w["seed"],
                     "design": w["design"], "redraws": int(info["redraws"]),
                     "theta_seed": 3001, "theta_box": [[0.5, 2.0], [0.02, 0.3], [0.3, 3.0]],
                     "theta_redraws": redraws},
        "points": points,
        "host": _host(),
    }
    out = os.path.join(HERE, "eval_n10k_oracle.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", out, flush=True)


def main():
    oracle.build(force=False)
    which = sys.argv[1:] or ["n20k", "n10k"]
    for wname in which:
        {"n20k": n20k, "n10k": n10k}[wname]()


if __name__ == "__main__":
    main()
