"""Writes converged_refs.json: the oracle's optimal values of the pendulum workload (N = 10,
seeds 0-2, instance parameters from workloads.instance_params) solved to max KKT residual
1e-8.  Calls only the oracle; the GPU parity tests compare converged device solutions with
these values.

Run from the repository root:  python tests/golden/make_converged_refs.py
"""
from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    oracle.build(force=False)
    out = {"what": "oracle sGS-ADMM (Algorithm 1, FP64) run to max(eta_p, eta_d, eta_g) <= 1e-8",
           "family": "pendulum", "N": 10, "cases": []}
    for seed in (0, 1, 2):
        prm = W.instance_params(W.PENDULUM, seed)
        sdp = oracle.relax(W.PENDULUM, 10, prm)
        r = oracle.admm_solve(sdp, tol=1e-8, maxiter=200000)
        out["cases"].append({"seed": seed, "params": [float(v) for v in prm], "pobj": r["pobj"],
                             "dobj": r["dobj"], "iters": int(r["iters"]),
                             "eta": max(r["eta_p"], r["eta_d"], r["eta_g"])})
        print(out["cases"][-1], flush=True)
    with open(os.path.join(HERE, "converged_refs.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
