"""Writes the oracle's results on the full-size workloads, sampled, for the
GPU parity tests that run those workloads at their real size:

  fk_1024_rk4_<T>.npz          Fenton-Karma 1024^2, 9-point, RK4: the state
                               after T = 1000 steps.
  bocf_2048_aniso_rk4_<T>.npz  Bueno-Orovio 2048^2, anisotropic flux form,
                               RK4: the state after T = 200 and 1000 steps
                               (one run, saved at both horizons).
  fk_ensemble_jvp_<n>_<T>.npz  the first Fenton-Karma ensemble member of
                               each grid size n in {256, 384, 512, 768}: state
                               and exact tangent after T = 200 RK4 steps (the
                               oracle's complex-step JVP along the member's
                               seeded unit direction).

Each file holds the sampled cells (16 x 16 windows at the four corners, the
four edge midpoints and the centre, the middle row, the middle column and
1024 seeded random cells) as index arrays ``iy``, ``ix`` and values
``state`` (and ``tangent``) of shape (n_fields, n_cells), plus the per-field
maximum of |value| over the WHOLE grid (``state_max``, ``tangent_max``), the
denominator of the relative L-infinity error.

Calls only the oracle and the seeded input generators.  Single-threaded
NumPy: about 11 CPU-minutes for the Fenton-Karma run, 10 for the ensemble
members and 2.3 CPU-hours for the Bueno-Orovio run (8 s per step).

    python tests/golden/make_fullsize_goldens.py fk|bocf|ensemble
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

WINDOW = 16
N_RANDOM = 1024
SAMPLE_SEED = 97


def sample_cells(nx: int, ny: int):
    """(iy, ix) of the sampled cells, de-duplicated, in a fixed order."""
    cells = []
    for y0 in (0, ny // 2 - WINDOW // 2, ny - WINDOW):
        for x0 in (0, nx // 2 - WINDOW // 2, nx - WINDOW):
            for j in range(y0, y0 + WINDOW):
                for i in range(x0, x0 + WINDOW):
                    cells.append((j, i))
    cells += [(ny // 2, i) for i in range(nx)]
    cells += [(j, nx // 2) for j in range(ny)]
    rng = np.random.default_rng(SAMPLE_SEED)
    cells += list(zip(rng.integers(0, ny, N_RANDOM).tolist(), rng.integers(0, nx, N_RANDOM).tolist()))
    seen, out = set(), []
    for c in cells:
        if c not in seen:
            seen.add(c)
            out.append(c)
    iy = np.array([c[0] for c in out], dtype=np.int32)
    ix = np.array([c[1] for c in out], dtype=np.int32)
    return iy, ix


def path(name: str, nsteps: int) -> str:
    return os.path.join(HERE, f"{name}_{nsteps}.npz")


def save(name: str, w: dict, nsteps: int, state, tangent=None, extra=None) -> None:
    iy, ix = sample_cells(w["nx"], w["ny"])
    meta = {"workload": name, "model": w["model"], "stencil": w["stencil"], "scheme": w["scheme"],
            "nx": w["nx"], "ny": w["ny"], "dt": w["dt"], "nsteps": nsteps, "seed": w["seed"],
            "window": WINDOW, "n_random": N_RANDOM, "sample_seed": SAMPLE_SEED}
    meta.update(extra or {})
    arrs = {"iy": iy, "ix": ix,
            "state": np.stack([a[iy, ix] for a in state]),
            "state_max": np.array([float(np.max(np.abs(a))) for a in state]),
            "meta": np.array(json.dumps(meta))}
    if tangent is not None:
        arrs["tangent"] = np.stack([a[iy, ix] for a in tangent])
        arrs["tangent_max"] = np.array([float(np.max(np.abs(a))) for a in tangent])
    np.savez_compressed(path(name, nsteps), **arrs)
    print(f"wrote {path(name, nsteps)} ({len(iy)} cells) {json.dumps(meta)}", flush=True)


def load(name: str, nsteps: int) -> dict:
    """The stored sample as a dict of arrays (``meta`` parsed from JSON)."""
    with np.load(path(name, nsteps), allow_pickle=False) as f:
        out = {k: f[k] for k in f.files}
    out["meta"] = json.loads(str(out["meta"]))
    return out


def oracle_problem(w: dict):
    return oracle.Problem.from_workload(w, params=ri.params_array(w["model"]))


def run_forward(name: str, horizons) -> None:
    w = ri.workload(name)
    po = oracle_problem(w)
    z = ri.initial_condition(w)
    done = 0
    t0 = time.time()
    for T in horizons:
        z = oracle.step(po, z, T - done)
        done = T
        save(name, w, T, z, extra={"oracle_seconds": round(time.time() - t0, 1)})


def run_ensemble(nsteps: int) -> None:
    members = ri.fk_batch_workloads(nsteps=nsteps)
    for n in ri.FK_BATCH_SIZES:
        w = next(m for m in members if m["nx"] == n)
        po = oracle_problem(w)
        z0 = ri.initial_condition(w)
        v = ri.direction(3, n, n, w["direction_seed"])
        t0 = time.time()
        zT, dz = oracle.jvp(po, z0, v, nsteps)
        save(f"fk_ensemble_jvp_{n}", w, nsteps, zT, dz,
             extra={"direction_seed": w["direction_seed"], "oracle_seconds": round(time.time() - t0, 1)})


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["fk", "bocf", "ensemble"])
    args = ap.parse_args()
    if args.which == "fk":
        run_forward("fk_1024_rk4", [1000])
    elif args.which == "bocf":
        run_forward("bocf_2048_aniso_rk4", [200, 1000])
    else:
        run_ensemble(200)


if __name__ == "__main__":
    main()
