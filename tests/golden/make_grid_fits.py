"""Writes grid_fits_n10k_oracle.json: the oracle's Fisher-BT fit (Algorithm 1
from the L9 start of Table 1, the paper's simulation bounds) for each setting
of the 3 x 3 simulation grid on the 100 x 100 jittered grid (n = 10,000):
sigma2 = 1, beta in {0.03, 0.1, 0.3}, nu in {0.5, 1.0, 2.5}, one realisation
per setting.  The file is rewritten after every setting, so a partial run
leaves the settings it finished.

It calls only the oracle and the seeded input generator; a setting takes from
tens of minutes (a converging fit) to hours (a fit that exhausts the scoring
budget and ends with Nelder-Mead).

    python tests/golden/make_grid_fits.py [i_beta,i_nu ...]
"""
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

OUT = os.path.join(HERE, "grid_fits_n10k_oracle.json")
# the settings whose fits converge first, the three that end in Nelder-Mead last
ORDER = [(0, 0), (1, 0), (2, 0), (1, 1), (2, 1), (0, 2), (0, 1), (1, 2), (2, 2)]


def fit_setting(ib, inu):
    w = synth.grid_workload(ib, inu)
    locs, z, info = synth.dataset(w["n"], w["theta_true"], w["seed"], design=w["design"])
    ev = oracle.OracleEvaluator(locs, z)
    t0 = time.perf_counter()
    iterates = []

    def cb(it, th, ll, g, fi):
        iterates.append({"iter": int(it), "theta": np.asarray(th).tolist(), "loglik": float(ll)})
        print("  [%6.0f s] iterate %d theta=%s loglik=%r" % (time.perf_counter() - t0, it,
                                                          np.round(th, 8).tolist(), float(ll)),
              flush=True)

    lo, hi = (0.01, 0.01, 0.01), (5.0, 5.0, 2.0)
    r = oracle.fisher_bt(ev, lo=lo, hi=hi, callback=cb)
    return {
        "i_beta": ib, "i_nu": inu, "theta_true": list(w["theta_true"]), "seed": w["seed"],
        "redraws": int(info["redraws"]), "bounds": {"lower": list(lo), "upper": list(hi)},
        "theta": np.asarray(r["theta"]).tolist(), "loglik": float(r["loglik"]),
        "score": np.asarray(r["score"]).tolist(),
        "n_loglik_calls": int(r["n_loglik_calls"]), "n_grad_calls": int(r["n_grad_calls"]),
        "n_iter": int(r["n_iter"]), "converged": bool(r["converged"]),
        "used_nelder_mead": bool(r["used_nelder_mead"]), "iterates": iterates,
        "host_seconds": time.perf_counter() - t0,
    }


def main():
    oracle.build(force=False)
    todo = ORDER
    if len(sys.argv) > 1:
        todo = [tuple(int(v) for v in a.split(",")) for a in sys.argv[1:]]
    rec = {"what": "oracle Fisher-BT fits (Algorithm 1, L9 start of Table 1, simulation bounds) "
                   "on the 3 x 3 simulation grid, n = 10,000 jittered grid", "fits": []}
    if os.path.exists(OUT):
        with open(OUT) as f:
            rec = json.load(f)
    done = {(f["i_beta"], f["i_nu"]) for f in rec["fits"]}
    for ib, inu in todo:
        if (ib, inu) in done:
            continue
        print("setting beta index %d, nu index %d" % (ib, inu), flush=True)
        rec["fits"].append(fit_setting(ib, inu))
        with open(OUT, "w") as f:
            json.dump(rec, f, indent=1)
        print("wrote %s (%d settings)" % (OUT, len(rec["fits"])), flush=True)


if __name__ == "__main__":
    main()
