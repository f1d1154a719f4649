"""Writes fit_n20k_oracle.json: the oracle's Fisher-BT fit (Algorithm 1 from the
L9 start of Table 1, the paper's simulation bounds) on the 20,000-point
benchmark field, for the full-size fit parity test.

It calls only the oracle and the seeded input generator; one run takes a few
hours of host time (about 70 oracle calls, each with dense n x n work).

    python tests/golden/make_fit_n20k.py [--n 20000]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import synth  # noqa: E402


class LoggedEvaluator(oracle.OracleEvaluator):
    """The oracle evaluator with one progress line per call."""

    def __init__(self, locs, z):
        super().__init__(locs, z)
        self.t0 = time.perf_counter()
        self.calls = 0

    def _log(self, what, theta, v):
        self.calls += 1
        print("[%7.0f s] call %d %s theta=%s -> %r" % (time.perf_counter() - self.t0, self.calls,
                                                       what, np.round(theta, 9).tolist(), v),
              flush=True)

    def loglik(self, theta):
        v = super().loglik(theta)
        self._log("loglik", theta, v)
        return v

    def evaluate(self, theta):
        r = super().evaluate(theta)
        self._log("evaluate", theta, r[0])
        return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--out", default=os.path.join(HERE, "fit_n20k_oracle.json"))
    args = ap.parse_args()
    oracle.build(force=False)
    w = dict(synth.WORKLOADS["n20k"])
    locs, z, info = synth.dataset(args.n, w["theta_true"], w["seed"])
    lo, hi = (0.01, 0.01, 0.01), (5.0, 5.0, 2.0)
    ev = LoggedEvaluator(locs, z)
    iterates = []

    def cb(it, th, ll, g, fi):
        iterates.append({"iter": int(it), "theta": np.asarray(th).tolist(), "loglik": float(ll),
                         "score": np.asarray(g).tolist()})

    t0 = time.perf_counter()
    r = oracle.fisher_bt(ev, lo=lo, hi=hi, callback=cb)
    dt = time.perf_counter() - t0
    rec = {
        "what": "oracle Fisher-BT fit (Algorithm 1, L9 start of Table 1, simulation bounds)",
        "workload": {"n": args.n, "theta_true": list(w["theta_true"]), "seed": w["seed"],
                     "design": w["design"], "redraws": int(info["redraws"])},
        "bounds": {"lower": list(lo), "upper": list(hi)},
        "theta": np.asarray(r["theta"]).tolist(),
        "loglik": float(r["loglik"]),
        "score": np.asarray(r["score"]).tolist(),
        "n_loglik_calls": int(r["n_loglik_calls"]),
        "n_grad_calls": int(r["n_grad_calls"]),
        "n_iter": int(r["n_iter"]),
        "converged": bool(r["converged"]),
        "used_nelder_mead": bool(r["used_nelder_mead"]),
        "iterates": iterates,
        "host_seconds": dt,
    }
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", args.out, "theta", rec["theta"], "in %.0f s" % dt, flush=True)


if __name__ == "__main__":
    main()
