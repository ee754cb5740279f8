"""Writes adjoint_barkley_1024_rk4_<T>_projections.json: the oracle's gradient
of L = dx^2 sum u(T)^2 for the Barkley 1024^2 RK4 adjoint workload
(checkpoints every 64; T = the workload's 4000 steps, or --nsteps), projected
on seeded unit directions.

Calls only the oracle and the seeded input generators.  Single-threaded NumPy:
about 30 minutes on one core for 1000 steps, two hours for 4000.

    python tests/golden/make_adjoint_projections.py [--nsteps T]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import oracle  # noqa: E402
import rd_inputs as ri  # noqa: E402

WORKLOAD = "barkley_1024_rk4_adjoint"
SEEDS = list(range(5000, 5008))


def out_path(nsteps: int) -> str:
    return os.path.join(HERE, f"adjoint_barkley_1024_rk4_{nsteps}_projections.json")


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--nsteps", type=int, default=None)
    args = ap.parse_args()
    w = ri.workload(WORKLOAD)
    if args.nsteps:
        w["nsteps"] = args.nsteps
    po = oracle.Problem.from_workload(w, params=ri.params_array(w["model"]))
    z0 = ri.initial_condition(w)
    t0 = time.time()
    zT = oracle.step(po, z0, w["nsteps"])
    lam = [2.0 * w["dx"] ** 2 * zT[0], np.zeros_like(zT[1])]
    g = oracle.vjp(po, z0, lam, w["nsteps"], checkpoint_every=w["checkpoint_every"])
    proj = []
    for seed in SEEDS:
        v = ri.direction(2, w["nx"], w["ny"], seed)
        proj.append(sum(float(np.sum(a * b)) for a, b in zip(g, v)))
    rec = {
        "workload": WORKLOAD,
        "nsteps": w["nsteps"],
        "checkpoint_every": w["checkpoint_every"],
        "loss": "dx^2 * sum(u(T)^2); cotangent (2 dx^2 u(T), 0)",
        "direction_seeds": SEEDS,
        "projections": proj,
        "max_abs_gradient": max(float(np.max(np.abs(a))) for a in g),
        "loss_value": float(np.sum(zT[0] ** 2) * w["dx"] ** 2),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(out_path(w["nsteps"]), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
