"""Benchmark: FP64 cell-updates/s of the fused explicit step on one MI355X.

Headline workload: the Bueno-Orovio 4-variable model (Eq. 5) on a 2048 x 2048
grid, anisotropic diffusion tensor (D_par = 0.001171, D_perp = D_par / 4
cm^2/ms, fibre angle rotating linearly from -60 to +60 degrees across x) in
conservative flux form, classical RK4, dx = 0.025 cm, dt = 0.05 ms, seeded
multi-spiral initial condition -- the largest single-grid workload.  One
benchmark "step" is one RK4 time step of the whole grid (one fused kernel
launch).  Inputs are resident in HBM before the timed region; the state is
advanced in place.  The K timed steps are taken as REPEATS windows of exactly
K steps each (HIP events on the launch stream, synchronised on both sides);
the reported rate is the median window, with the spread.

Prints one JSON line (see the keys below).  --gpus N with N > 1 exits: this
build runs on a single GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12           # bytes/s, MI355X HBM3E
# Arrays streamed per field and cell by one RK4 step of the 3-D stage kernels:
# stage 1 reads z, writes k1; stages 2 and 3 read z and k_{s-1}, write k_s;
# stage 4 reads z, k1, k2, k3 and writes the new state: 2 + 3 + 3 + 5.
STAGE3_RK4_FIELDS = 13
FP64_VECTOR_PEAK = 78.6e12  # flop/s, MI355X FP64 vector (FMA = 2 flops)
KERNEL_SOURCES = ["paper_1309_1720_amd/csrc/rd_device.h", "paper_1309_1720_amd/csrc/rd_sweep.h"]
# Algorithmic FP64 operations per Fenton-Karma RK4 cell-update, counted from the
# equations as evaluated (9-point stencil 11, reaction 51 + one exp, stage
# updates; each add, multiply, divide and exp counts 1).
FK_RK4_FLOPS = 295
# Algorithmic HBM bytes per cell-update of one step: read and write the state
# once, 2 n_v 8 bytes.
B_ALG = {"diffusion": 16, "barkley": 32, "fhn": 32, "fk": 48, "bocf": 64}
HEADLINE = "bocf_2048_aniso_rk4"
HEADLINE_NAME = "bueno_orovio_2048x2048_lap9_aniso_rk4"
REPEATS = 5
MODEL_NAMES = {"diffusion": "diffusion", "barkley": "Barkley", "fhn": "FitzHugh-Nagumo", "fk": "Fenton-Karma",
               "bocf": "Bueno-Orovio (epicardial)"}


def counters_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"fwd_{workload}_counters.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_counters(workload: str):
    """The committed counter record of ``workload``'s fused step if it was
    taken on the current kernel sources, else None."""
    path = counters_file(workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        c = json.load(fh)
    return c if c.get("kernel_sha") == kernel_hash() else None


def measured_counters(workload: str, cells: int, tile_rows: int):
    """The committed counter record, if it was taken on the current kernel
    sources, this grid and the band height in use; else None."""
    c = committed_counters(workload)
    if c is None or c.get("cells") != cells or c.get("tile_rows") != tile_rows:
        return None
    return c


# Vector-instruction issue capacity: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (a wave64 VALU instruction, FP64 included, occupies a SIMD for 4 cycles).
VALU_LANE_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9


def valu_issue(c, launch_s: float):
    """Lane-instructions per second of the fused step (committed counter
    record x the live launch time) against the issue capacity."""
    if not c or "valu_instructions_per_launch" not in c:
        return None
    achieved = c["valu_instructions_per_launch"] * 64 / launch_s
    return {"achieved": achieved / 1e12, "peak": VALU_LANE_ISSUE_PEAK / 1e12, "unit": "T lane-instr/s",
            "frac": achieved / VALU_LANE_ISSUE_PEAK,
            "lane_instructions_per_cell_update": c["lane_instructions_per_cell_update"]}


def windows(torch, stream, fn, reps: int = REPEATS) -> list:
    """Device seconds of fn() between two events on ``stream``, ``reps``
    windows, each synchronised on both sides."""
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / 1e3)
    return out


def median(xs):
    ys = sorted(xs)
    n = len(ys)
    return ys[n // 2] if n % 2 else 0.5 * (ys[n // 2 - 1] + ys[n // 2])


def window_stats(secs, steps: int) -> dict:
    med = median(secs)
    return {"windows": len(secs), "steps_per_window": steps,
            "us_per_step_median": med / steps * 1e6, "us_per_step_min": min(secs) / steps * 1e6,
            "us_per_step_max": max(secs) / steps * 1e6, "spread": (max(secs) - min(secs)) / med}


def forward_run(rd, torch, dev, name: str, steps: int, warmup: int, reps: int = REPEATS,
                tile_rows: int = 0, **over):
    """Times ``reps`` windows of exactly ``steps`` fused steps of workload
    ``name`` (state resident on the device, advanced in place) after
    ``warmup`` untimed steps.  Returns (record, final state)."""
    import rd_inputs as ri
    w = ri.workload(name, **over)
    model = w["model"]
    cells = w["nx"] * w["ny"]
    params = ri.params_array(model)
    z = [torch.from_numpy(a).to(dev) for a in ri.initial_condition(w)]
    if tile_rows:
        rd.set_tile_rows(tile_rows)
    try:
        p = rd.Problem.from_workload(w, params, nsteps=max(warmup, 1), checkpoint_every=0)
        rd.step(p, z)   # warm-up; the first call tunes the plan
        torch.cuda.synchronize()
        p.nsteps = steps
        stream = torch.cuda.current_stream(dev)
        secs = windows(torch, stream, lambda: rd.step(p, z), reps)
        variant, rows = rd.get_plan(p, "step")
        k = rd.get_steps_per_launch(p)
    finally:
        if tile_rows:
            rd.set_tile_rows(0)
    st = window_stats(secs, steps)
    sec = median(secs)
    launch_s = sec / steps * k
    b_alg = B_ALG[model]
    rec = {"workload": name, "nx": w["nx"], "ny": w["ny"], "model": model, "stencil": w["stencil"],
           "scheme": w["scheme"], "rate": cells * steps / sec, "us_per_step": st["us_per_step_median"],
           "timing": st, "plan": [variant, rows], "steps_per_launch": k,
           "hbm_bytes_per_cell_update": b_alg, "algorithmic_bytes_per_launch": b_alg * cells * k,
           "avg_launch_us": launch_s * 1e6, "hbm_frac": b_alg * cells * steps / sec / HBM_PEAK}
    c = measured_counters(name, cells, rows) if variant == "sweep" else None
    rec["traffic"] = c["hbm_bytes_per_launch"] if c else None
    rec["valu_issue"] = valu_issue(c, launch_s)
    return rec, z


def cpu_baseline(w, params, seconds: float, label: str):
    """The oracle as it stands, on the host, over a bounded number of steps
    of the same workload (whole grid)."""
    import oracle
    import rd_inputs as ri
    po = oracle.Problem.from_workload(w, params=params)
    z = ri.initial_condition(w)
    z = oracle.step(po, z, 1)  # warm-up
    n, t0 = 0, time.perf_counter()
    while True:
        z = oracle.step(po, z, 1)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 1000:
            break
    rate = w["nx"] * w["ny"] * n / el
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), cpu)
    except OSError:
        pass
    return {"value": rate, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "host_cpu": cpu, "host_threads": os.cpu_count(),
            "sample": f"{n} {w['scheme'].upper()} steps of the whole {w['nx']}x{w['ny']} {label} grid "
                      f"after one warm-up step (NumPy, single thread), {el:.1f} s"}


def jvp_report(rd, torch, w, params, z0_np, fwd_ms, steps, dev):
    """Exact tangent-linear JVP (rd_jvp) against central finite differences of
    two forward runs, on the same grid: cost per step and accuracy."""
    import numpy as np
    import rd_inputs as ri
    nx, ny = w["nx"], w["ny"]
    v_np = ri.direction(3, nx, ny, 4100)
    stream = torch.cuda.current_stream(dev)
    # cost: jvp steps timed like the forward
    z = [torch.from_numpy(a).to(dev) for a in z0_np]
    v = [torch.from_numpy(a).to(dev) for a in v_np]
    p = rd.Problem.from_workload(w, params, nsteps=20)
    rd.jvp(p, z, v)
    p.nsteps = steps
    jvp_ms = median(windows(torch, stream, lambda: rd.jvp(p, z, v), 3)) * 1e3 / steps
    jvp_rows = rd.get_tile_rows(p, "jvp")
    # algorithmic bytes: read and write the state and its tangent once
    jvp_bytes = 4 * len(z0_np) * 8
    # accuracy over a short horizon: FD error relative to the exact JVP
    horizon = 100
    p = rd.Problem.from_workload(w, params, nsteps=horizon)
    z = [torch.from_numpy(a).to(dev) for a in z0_np]
    v = [torch.from_numpy(a).to(dev) for a in v_np]
    rd.jvp(p, z, v)
    jv = torch.cat([t.flatten() for t in v])
    # v has unit norm over all 3 nx ny entries, so eps * v perturbs a cell by
    # about eps / 1800: the range reaches the truncation side of the V-curve
    errs = {}
    for k in range(9, -1, -1):
        eps = 10.0 ** (-k)
        zp = [torch.from_numpy(a + eps * b).to(dev) for a, b in zip(z0_np, v_np)]
        zm = [torch.from_numpy(a - eps * b).to(dev) for a, b in zip(z0_np, v_np)]
        rd.step(p, zp)
        rd.step(p, zm)
        fd = (torch.cat([t.flatten() for t in zp]) - torch.cat([t.flatten() for t in zm])) / (2 * eps)
        errs[f"{eps:.0e}"] = float(torch.linalg.norm(fd - jv) / torch.linalg.norm(jv))
    return {"ms_per_step": jvp_ms, "over_forward": jvp_ms / fwd_ms, "tile_rows": jvp_rows,
            "hbm_bytes_per_cell_update": jvp_bytes,
            "hbm_frac": nx * ny * jvp_bytes / (jvp_ms * 1e-3) / HBM_PEAK,
            "fd_jvp_ms_per_step": 2 * fwd_ms, "fd_rel_err_by_eps": errs,
            "fd_best_rel_err": min(errs.values()), "horizon_steps": horizon,
            "timed_steps": steps}


def _timed(torch, stream, fn, reps=1):
    """Device time of fn() between two events on `stream` (best of `reps`)."""
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    return best


def ensemble_report(rd, torch, dev, nsteps: int):
    """The ensemble workload as specified: 64 Fenton-Karma instances (16 each
    of 256^2 .. 768^2) with seeded unit directions, the forward flow plus the
    exact JVP over ``nsteps`` RK4 steps (T = 200 ms at 2000 steps) in one
    batched call per launch sequence, timed end to end; forward-only and
    per-instance calls for comparison; a graph replay; and central
    finite-difference JVPs at the same horizon for eps = 1e-9 .. 1e-5."""
    import rd_inputs as ri
    stream = torch.cuda.current_stream(dev)
    ws = ri.fk_batch_workloads(nsteps=2)
    params = ri.params_array("fk")
    probs = [rd.Problem.from_workload(x, params) for x in ws]
    z0 = [ri.fk_ic(x["nx"], x["ny"], x["seed"]) for x in ws]
    v0 = [ri.direction(3, x["nx"], x["ny"], x["direction_seed"]) for x in ws]
    to_dev = lambda zs: [[torch.from_numpy(a).to(dev) for a in z] for z in zs]
    fields, tans = to_dev(z0), to_dev(v0)
    rd.step_batched(probs, fields, tans)      # first calls tune the band height
    rd.step_batched(probs, fields, None)
    for q, f, t in zip(probs, fields, tans):
        rd.jvp(q, f, t)
    torch.cuda.synchronize()
    cells = sum(x["nx"] * x["ny"] for x in ws)
    out = {"members": len(ws), "cells": cells}
    # short windows: per-step cost of the batched JVP, forward and per-instance calls
    n = 20
    for q in probs:
        q.nsteps = n
    sec_b = median(windows(torch, stream, lambda: rd.step_batched(probs, fields, tans)))
    sec_f = median(windows(torch, stream, lambda: rd.step_batched(probs, fields, None)))

    def per_instance():
        for q, f, t in zip(probs, fields, tans):
            rd.jvp(q, f, t)
    sec_s = median(windows(torch, stream, per_instance, 3))
    gstream = torch.cuda.Stream(dev)
    gstream.wait_stream(stream)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(gstream):
        with torch.cuda.graph(graph, stream=gstream):
            rd.step_batched(probs, fields, tans)
    stream.wait_stream(gstream)
    sec_g = median(windows(torch, stream, graph.replay, 3))
    del graph
    out.update({"window_steps": n, "rate_jvp": cells * n / sec_b, "rate_forward": cells * n / sec_f,
                "jvp_over_forward": sec_b / sec_f, "per_instance_calls_over_batched": sec_s / sec_b,
                "rate_jvp_graph_replay": cells * n / sec_g, "hbm_frac_jvp": 96 * cells * n / sec_b / HBM_PEAK})
    # the whole flow over the horizon, from the seeded initial states
    for q in probs:
        q.nsteps = nsteps
    fields, tans = to_dev(z0), to_dev(v0)
    sec_T = windows(torch, stream, lambda: rd.step_batched(probs, fields, tans), 1)[0]
    fwd = to_dev(z0)
    sec_Tf = windows(torch, stream, lambda: rd.step_batched(probs, fwd, None), 1)[0]
    if not all(bool(torch.equal(a, b)) for fa, fb in zip(fields, fwd) for a, b in zip(fa, fb)):
        raise RuntimeError("ensemble: the JVP run's state differs from the forward run's")
    del fwd
    jv = [torch.cat([t.flatten() for t in tl]) for tl in tans]
    fd_err = {}
    for k in range(9, 4, -1):
        eps = 10.0 ** (-k)
        zp = to_dev([[a + eps * b for a, b in zip(z, v)] for z, v in zip(z0, v0)])
        zm = to_dev([[a - eps * b for a, b in zip(z, v)] for z, v in zip(z0, v0)])
        rd.step_batched(probs, zp, None)
        rd.step_batched(probs, zm, None)
        errs = []
        for i in range(len(ws)):
            fd = (torch.cat([t.flatten() for t in zp[i]]) - torch.cat([t.flatten() for t in zm[i]])) / (2 * eps)
            errs.append(float(torch.linalg.norm(fd - jv[i]) / torch.linalg.norm(jv[i])))
        fd_err[f"{eps:.0e}"] = {"median": median(errs), "max": max(errs), "min": min(errs)}
        del zp, zm
    best = min(fd_err, key=lambda e: fd_err[e]["median"])
    out.update({"horizon_steps": nsteps, "horizon_ms": nsteps * ws[0]["dt"],
                "flow_and_jvp_seconds": sec_T, "forward_flow_seconds": sec_Tf,
                "flow_jvp_over_forward": sec_T / sec_Tf,
                "rate_jvp_horizon": cells * nsteps / sec_T,
                "fd_jvp_seconds": 2 * sec_Tf,
                "fd_rel_err_by_eps": fd_err, "fd_best_eps": best,
                "fd_best_median_rel_err": fd_err[best]["median"]})
    return out


def other_workloads(rd, torch, dev, only=None, steps: int = 200):
    """Timings of the other workloads (rates in cell-updates/s, device time,
    median of REPEATS windows where a window is cheap); ``only`` names one of
    them to run alone."""
    import rd_inputs as ri
    stream = torch.cuda.current_stream(dev)
    out = {}

    if only in (None, "fk_1024_rk4"):
        # Fenton-Karma 1024^2, 9-point, RK4 (the workload of the tangent record)
        rec, _ = forward_run(rd, torch, dev, "fk_1024_rk4", steps, 20)
        rec["roofline_alu"] = {"bound": "alu", "achieved": FK_RK4_FLOPS * rec["rate"] / 1e12,
                               "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                               "frac": FK_RK4_FLOPS * rec["rate"] / FP64_VECTOR_PEAK,
                               "flops_per_cell_update": FK_RK4_FLOPS}
        out["fk_1024_rk4"] = rec

    if only in (None, "barkley_128_euler_1000"):
        # Barkley 128^2, 5-point, Euler, 1000 steps (whole run)
        w = ri.workload("barkley_128_euler")
        z = [torch.from_numpy(a).to(dev) for a in ri.initial_condition(w)]
        p = rd.Problem.from_workload(w, ri.params_array("barkley"), nsteps=20)
        rd.step(p, z)
        p.nsteps = w["nsteps"]
        sec = median(windows(torch, stream, lambda: rd.step(p, z)))
        # the same 1000 steps captured once in a HIP graph and replayed (no
        # per-launch host overhead)
        gstream = torch.cuda.Stream(dev)
        gstream.wait_stream(stream)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(gstream):
            with torch.cuda.graph(graph, stream=gstream):
                rd.step(p, z)
        stream.wait_stream(gstream)
        sec_g = median(windows(torch, stream, graph.replay))
        out["barkley_128_euler_1000"] = {"seconds": sec, "rate": 128 * 128 * w["nsteps"] / sec,
                                         "steps_per_launch": rd.get_steps_per_launch(p),
                                         "us_per_step": sec / w["nsteps"] * 1e6,
                                         "us_per_step_graph_replay": sec_g / w["nsteps"] * 1e6,
                                         "rate_graph_replay": 128 * 128 * w["nsteps"] / sec_g,
                                         "hbm_frac": 32 * 128 * 128 * w["nsteps"] / sec / HBM_PEAK}
        del graph

    if only in (None, "fhn_256_rk4_1000"):
        # FitzHugh-Nagumo 256^2 (Eq. 3, u and v diffusive), 9-point, RK4, 1000 steps
        w = ri.workload("fhn_256_rk4")
        z = [torch.from_numpy(a).to(dev) for a in ri.initial_condition(w)]
        p = rd.Problem.from_workload(w, ri.params_array("fhn"), nsteps=8)
        rd.step(p, z)
        p.nsteps = w["nsteps"]
        sec = median(windows(torch, stream, lambda: rd.step(p, z)))
        cells = w["nx"] * w["ny"]
        out["fhn_256_rk4_1000"] = {"seconds": sec, "rate": cells * w["nsteps"] / sec,
                                   "us_per_step": sec / w["nsteps"] * 1e6,
                                   "steps_per_launch": rd.get_steps_per_launch(p),
                                   "plan": list(rd.get_plan(p, "step")),
                                   "hbm_frac": 32 * cells * w["nsteps"] / sec / HBM_PEAK}

    if only in (None, "fk_4096_rk4_beyond_llc"):
        # Beyond the 256 MB last-level cache: Fenton-Karma 4096^2 (3 x 128 MiB per
        # state), the same scheme, so the traffic really goes to HBM.
        rec, z = forward_run(rd, torch, dev, "fk_1024_rk4", 20, 2, reps=3, nx=4096, ny=4096)
        rec["workload"] = "fk_4096_rk4_beyond_llc"
        out["fk_4096_rk4_beyond_llc"] = rec
        del z

    if only in (None, "barkley_8192_rk4_beyond_llc"):
        # HBM-bound 2-D probe beyond the 256 MB last-level cache: Barkley
        # 8192^2 (1 GiB per state), 5-point, RK4, steps per launch tuned.
        rec, z = forward_run(rd, torch, dev, "barkley_1024_rk4_adjoint", 16, 4, reps=3, nx=8192, ny=8192)
        rec["workload"] = "barkley_8192_rk4_beyond_llc"
        out["barkley_8192_rk4_beyond_llc"] = rec
        del z

    if only in (None, "barkley_1024_rk4"):
        # the adjoint workload's forward step alone (no checkpoints)
        rec, _ = forward_run(rd, torch, dev, "barkley_1024_rk4_adjoint", steps, 20)
        out["barkley_1024_rk4"] = rec

    if only in (None, "fk_ensemble_64_jvp"):
        out["fk_ensemble_64_jvp"] = ensemble_report(rd, torch, dev, 2000)

    if only in (None, "newton_krylov_fhn_3_members_200_steps"):
        # Newton-Krylov fixed points of the 200-step FitzHugh-Nagumo flow for a
        # small ensemble (stable and unstable uniform states), exact vs FD JVPs
        import numpy as np
        from paper_1309_1720_amd import krylov
        fp = ri.FHN_PARAMS
        roots = sorted(r.real for r in np.roots([1.0, 0.0, -(1.0 - 1.0 / fp["a1"]), -fp["a0"] / fp["a1"]])
                       if abs(r.imag) < 1e-12)
        members = []
        for (nx, ny), u in (((96, 80), roots[0]), ((128, 96), roots[2]), ((160, 128), roots[0])):
            wk = ri.workload("fhn_256_rk4", nx=nx, ny=ny, nsteps=200)
            i = np.arange(nx)[None, :]
            j = np.arange(ny)[:, None]
            pat = np.cos(np.pi * (i + 0.5) / nx) * np.cos(2 * np.pi * (j + 0.5) / ny)
            v = (u - fp["a0"]) / fp["a1"]
            members.append((rd.Problem.from_workload(wk, ri.params_array("fhn")),
                            [torch.from_numpy(u + 0.01 * pat).to(dev), torch.from_numpy(v + 0.02 * pat).to(dev)]))
        nk = {}
        for kind in ("exact", "fd"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = krylov.newton_krylov([m[0] for m in members], [m[1] for m in members], tol=1e-13,
                                       max_newton=8, jvp=kind)
            torch.cuda.synchronize()
            nk[kind] = {"seconds": time.perf_counter() - t0, "residuals": res.residuals,
                        "krylov_iterations": res.krylov_iterations}
        out["newton_krylov_fhn_3_members_200_steps"] = nk

    if only in (None, "periodic_orbit_barkley_spirals"):
        # Newton-Krylov for the periodic orbits of rotating Barkley spirals
        # (64^2 and 128^2, RK4, N = 160 steps per period, periods unknown),
        # exact vs central-difference JVPs, from spirals settled for 300 time
        # units (the period guess is the return time nearest to the state).
        import numpy as np
        from paper_1309_1720_amd import krylov
        N = 160
        members = []
        for n in (64, 128):
            wk = ri.workload("barkley_128_euler", nx=n, ny=n, scheme="rk4")
            params = ri.params_array("barkley")
            z = [torch.from_numpy(a).to(dev) for a in ri.initial_condition(wk)]
            rd.step(rd.Problem.from_workload(wk, params, nsteps=int(round(300.0 / wk["dt"]))), z)
            z0 = [a.clone() for a in z]
            one = rd.Problem.from_workload(wk, params, nsteps=1)
            dist = []
            for _ in range(260):
                rd.step(one, z)
                dist.append(sum(float(torch.sum((a - b) ** 2)) for a, b in zip(z, z0)))
            nstar = 100 + int(np.argmin(dist[99:]))
            members.append((rd.Problem.from_workload(wk, params, nsteps=N), z0, nstar * wk["dt"]))
        po = {"members": ["barkley 64^2 rk4", "barkley 128^2 rk4"], "steps_per_period": N}
        for kind in ("exact", "fd"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = krylov.periodic_orbit([m[0] for m in members], [m[1] for m in members],
                                        [m[2] for m in members], tol=1e-10, jvp=kind)
            torch.cuda.synchronize()
            po[kind] = {"seconds": time.perf_counter() - t0, "residuals": res.residuals,
                        "krylov_iterations": res.krylov_iterations, "periods": res.periods}
        out["periodic_orbit_barkley_spirals"] = po

    if only in (None, "fk_256cube_lap27_rk4"):
        # 3-D: Fenton-Karma 256^3, 27-point, RK4 (20 of its 1000 steps), one
        # HBM-streaming launch per stage (STAGE3_RK4_FIELDS arrays per field and cell).
        w = ri.workload("fk_256cube_lap27_rk4")
        z = [torch.from_numpy(a).to(dev) for a in ri.initial_condition(w)]
        p = rd.Problem.from_workload(w, ri.params_array("fk"), nsteps=2)
        rd.step(p, z)
        n = 20
        p.nsteps = n
        sec = median(windows(torch, stream, lambda: rd.step(p, z), 3))
        cells = w["nx"] * w["ny"] * w["nz"]
        # tangent (exact JVP) over the same 20 steps
        v = [torch.from_numpy(a).to(dev) for a in ri.direction(3, w["nx"], w["ny"], 4200, nz=w["nz"])]
        pj = rd.Problem.from_workload(w, ri.params_array("fk"), nsteps=n)
        rd.jvp(pj, [t.clone() for t in z], [t.clone() for t in v])
        sec_jvp = _timed(torch, stream, lambda: rd.jvp(pj, z, v))
        del v
        # adjoint over the same 20 steps, checkpoints every 10
        p.checkpoint_every = 10
        ck = torch.empty(rd.checkpoint_count(p) * 3 * cells, dtype=torch.float64, device=dev)
        sec_ck = _timed(torch, stream, lambda: rd.step(p, z, ck))
        lam = [t.clone() for t in z]
        rd.vjp(p, ck, [t.clone() for t in z])
        sec_vjp = _timed(torch, stream, lambda: rd.vjp(p, ck, lam))
        stream_bytes = STAGE3_RK4_FIELDS * 3 * 8
        out["fk_256cube_lap27_rk4"] = {"steps": n, "rate": cells * n / sec, "us_per_step": sec / n * 1e6,
                                       "hbm_bytes_per_cell_update": B_ALG["fk"],
                                       "hbm_frac": B_ALG["fk"] * cells * n / sec / HBM_PEAK,
                                       "stage_stream_bytes_per_cell_update": stream_bytes,
                                       "stage_stream_frac": stream_bytes * cells * n / sec / HBM_PEAK,
                                       "jvp_us_per_step": sec_jvp / n * 1e6,
                                       "jvp_over_forward": sec_jvp / sec,
                                       "vjp_us_per_step": sec_vjp / n * 1e6,
                                       "vjp_over_forward_with_checkpoints": sec_vjp / sec_ck}
        del z, ck, lam

    if only in (None, "barkley_1024_rk4_adjoint_4000"):
        # Adjoint: Barkley 1024^2, RK4, 4000 steps, checkpoints every 64
        w = ri.workload("barkley_1024_rk4_adjoint")
        p = rd.Problem.from_workload(w, ri.params_array("barkley"))
        z = [torch.from_numpy(a).to(dev) for a in ri.initial_condition(w)]
        ck = torch.empty(rd.checkpoint_count(p) * 2 * w["nx"] * w["ny"], dtype=torch.float64, device=dev)
        warm = rd.Problem.from_workload(w, ri.params_array("barkley"), nsteps=2)
        rd.step(warm, [t.clone() for t in z])   # tunes the forward plan outside the timed region
        sec_fwd = _timed(torch, stream, lambda: rd.step(p, z, ck))
        lam = [(2.0 * w["dx"] ** 2) * z[0].clone(), torch.zeros_like(z[1])]
        sec_vjp = _timed(torch, stream, lambda: rd.vjp(p, ck, lam))
        cells = w["nx"] * w["ny"]
        out["barkley_1024_rk4_adjoint_4000"] = {
            "forward_seconds": sec_fwd, "vjp_seconds": sec_vjp, "vjp_over_forward": sec_vjp / sec_fwd,
            "forward_rate": cells * w["nsteps"] / sec_fwd, "forward_steps_per_launch": rd.get_steps_per_launch(p),
            "forward_hbm_frac": 32 * cells * w["nsteps"] / sec_fwd / HBM_PEAK,
            "forward_tile_rows": rd.get_tile_rows(p, "step"), "adjoint_tile_rows": rd.get_tile_rows(p, "vjp")}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=REPEATS,
                    help="timed windows of exactly --steps steps each; the median is reported")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--variant", choices=["sweep", "pipe"], default=None)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-jvp", action="store_true")
    ap.add_argument("--no-other-workloads", action="store_true")
    ap.add_argument("--only-workload", default=None,
                    help="run only this one of the other workloads and print its record")
    ap.add_argument("--workload", default=HEADLINE,
                    help="single-grid 2-D workload timed as the headline (profiling runs)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1309_1720_amd as rd
    import rd_inputs as ri

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only_workload:
        rec = other_workloads(rd, torch, dev, only=args.only_workload)
        if not rec:
            raise SystemExit(f"bench.py: unknown workload {args.only_workload!r}")
        print(json.dumps(rec))
        return

    name = args.workload
    w = ri.workload(name)
    if w["nz"] != 1:
        raise SystemExit(f"bench.py: {name} is not a 2-D workload")
    params = ri.params_array(w["model"])
    nx, ny = w["nx"], w["ny"]
    cells = nx * ny
    nv = ri.N_FIELDS[w["model"]]
    plan_source = "autotuned"
    tile_rows = args.tile_rows
    if tile_rows:
        plan_source = "--tile-rows"
    elif args.variant is None:
        # Run at the band height the committed counter profile was taken at
        # (when it matches the kernel sources), so that the traffic figure
        # describes this very launch.
        c = committed_counters(name)
        if c and c.get("cells") == cells:
            tile_rows = int(c["tile_rows"])
            plan_source = "band height of the committed counter profile"
    if args.variant:
        rd.set_kernel_variant(args.variant)
    t0 = time.perf_counter()
    rec, z = forward_run(rd, torch, dev, name, args.steps, args.warmup, args.repeats, tile_rows)
    wall = time.perf_counter() - t0
    if not all(bool(torch.isfinite(t).all()) for t in z):
        raise RuntimeError("non-finite state after the timed steps")
    del z
    if args.variant:
        rd.set_kernel_variant(None)
    if args.calibration_copy:
        # a plain elementwise copy of 2^26 doubles (512 MiB read + 512 MiB written)
        src = torch.rand(1 << 26, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0.0, out=dst)
        torch.cuda.synchronize()

    variant, rows = rec["plan"]
    launch_s = rec["avg_launch_us"] * 1e-6
    achieved = rec["algorithmic_bytes_per_launch"] / launch_s
    out = {
        "metric": "FP64 cell-updates/s",
        "value": rec["rate"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["us_per_step"] / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": HEADLINE_NAME if name == HEADLINE else name, "nx": nx, "ny": ny,
                   "model": MODEL_NAMES[w["model"]], "stencil": w["stencil"], "scheme": w["scheme"],
                   "dx": w["dx"], "dt": w["dt"], "D_par": w["D_par"], "D_perp": w["D_perp"],
                   "theta_deg": [round(math.degrees(w["theta0"])), round(math.degrees(w["theta1"]))],
                   "fields": nv},
        "timing": rec["timing"],
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK,
                     "traffic": rec["traffic"],
                     "algorithmic_bytes_per_launch": rec["algorithmic_bytes_per_launch"],
                     "avg_launch_us": rec["avg_launch_us"]},
        "valu_issue": rec["valu_issue"],
        "kernel_variant": variant,
        "tile_rows": rows,
        "plan_source": plan_source,
        "wall_s": wall,
    }
    if not args.no_jvp:
        wf = ri.workload("fk_1024_rk4")
        fk, _ = forward_run(rd, torch, dev, "fk_1024_rk4", 200, 20, 3)
        out["jvp"] = jvp_report(rd, torch, wf, ri.params_array("fk"), ri.initial_condition(wf),
                                fk["us_per_step"] / 1e3, 200, dev)
    if not args.no_other_workloads:
        out["other_workloads"] = other_workloads(rd, torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, params, args.cpu_seconds, MODEL_NAMES[w["model"]])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
