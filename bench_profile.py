"""Condense rocprofv3 output of the benchmark's fused step into the summaries
under profiles/ (text only) and the traffic record bench.py reads.

A 2-D workload's fused step (the headline Bueno-Orovio 2048^2 step, or the
Fenton-Karma 1024^2 one) from four runs of rocprofv3, each its own process,
from /tmp, with the band height T pinned:

    rocprofv3 --kernel-trace --stats --output-format csv -d OUT/stats -o fwd -- \
        python3 REPO/bench.py --steps 20 --warmup 5 --workload W --no-cpu-baseline --no-jvp \
        --no-other-workloads --variant sweep --repeats 1 --tile-rows T
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch -o fwd -- \
        (the same bench.py command) --calibration-copy
    (the same with --pmc WRITE_SIZE into OUT/write, and with the SQ counters
    below into OUT/sq, without the copy)

then:  python bench_profile.py --forward OUT W T

The 3-D stage kernels (Fenton-Karma 256^3, 27-point, RK4) from three runs of
`bench.py --only-workload fk_256cube_lap27_rk4` (kernel trace and stats,
FETCH_SIZE, WRITE_SIZE, each in OUT/stats, OUT/fetch, OUT/write):

       python bench_profile.py --stage3d OUT

The HBM-bound 2-D probe (Barkley 8192^2, 5-point, RK4, two steps per
launch) from the same three runs of `bench.py --only-workload
barkley_8192_rk4_beyond_llc` (OUT/stats with the kernel trace, OUT/fetch,
OUT/write):

       python bench_profile.py --barkley8192 OUT

The exact tangent step (rd_jvp) of the Fenton-Karma workload from three runs
of `bench.py --steps 200 --warmup 2 --no-cpu-baseline --no-other-workloads
--variant sweep --tile-rows T` (T the tangent's band height; OUT/stats,
OUT/fetch, OUT/write as above):

       python bench_profile.py --tangent OUT T
"""
from __future__ import annotations

import collections
import csv
import glob
import json
import os
import sys

import bench

HERE = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(HERE, "profiles")
CALIB = "CUDAFunctorOnSelf_add<double>"
CALIB_BYTES = 1 << 29  # 2^26 doubles read and the same written
SQ_COUNTERS = ["SQ_WAVES", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU",
               "SQ_WAIT_INST_ANY", "SQ_WAIT_ANY", "SQ_INSTS_SALU"]
BENCH_ARGS = "--no-cpu-baseline --no-jvp --no-other-workloads --variant sweep --repeats 1"


def _rows(root: str, pattern: str) -> list[dict]:
    out = []
    for f in sorted(glob.glob(os.path.join(root, "**", pattern), recursive=True)):
        with open(f) as fh:
            out += list(csv.DictReader(fh))
    return out


def _counters(root: str) -> dict:
    """(kernel, counter) -> mean value per dispatch."""
    agg = collections.defaultdict(list)
    for r in _rows(root, "*counter_collection.csv"):
        agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}


def _pick(counters: dict, needle: str, counter: str) -> float:
    vals = [v for (k, c), v in counters.items() if needle in k and c == counter]
    if len(vals) != 1:
        raise RuntimeError(f"expected one kernel matching {needle!r} with {counter}, found {len(vals)}")
    return vals[0]


MODEL_ID = {"diffusion": 0, "barkley": 1, "fk": 2, "bocf": 3, "fhn": 4}
STENCIL_ID = {"lap5": 5, "lap9": 9, "lap9_aniso": 10}
SCHEME_ID = {"euler": 1, "heun": 2, "rk4": 4}


def sweep_kernel(w: dict) -> str:
    """Name prefix of the fused state sweep of a 2-D workload."""
    return (f"rd::sweep_kernel<{MODEL_ID[w['model']]}, {STENCIL_ID[w['stencil']]}, "
            f"{SCHEME_ID[w['scheme']]}, 0, ")


def _trace_durations(root: str, needle: str) -> list:
    rows = [t for t in _rows(root, "*kernel_trace.csv") if needle in t["Kernel_Name"]]
    return [(int(t["End_Timestamp"]) - int(t["Start_Timestamp"])) / 1e3 for t in rows]


def main_forward(out: str, workload: str, tile_rows: int) -> None:
    """Kernel timings, HBM traffic and instruction counters of one 2-D
    workload's fused step, from four runs of bench.py with that workload as
    the headline at a pinned band height."""
    import rd_inputs as ri
    w = ri.workload(workload)
    cells = w["nx"] * w["ny"]
    alg = bench.B_ALG[w["model"]] * cells
    needle = sweep_kernel(w)
    args = f"--workload {workload} {BENCH_ARGS} --tile-rows {tile_rows}"
    cmd = lambda extra, steps: (f"cd /tmp && rocprofv3 {extra} --output-format csv -d <out> -o fwd -- "
                                f"python3 <repo>/bench.py --steps {steps} --warmup 400 {args}")
    title = f"{w['model']} {w['nx']}x{w['ny']}, {w['stencil']}, {w['scheme']}"

    stats = _rows(os.path.join(out, "stats"), "*kernel_stats.csv")
    row = [r for r in stats if needle in r["Name"]]
    if len(row) != 1:
        raise RuntimeError(f"expected one kernel matching {needle!r}, found {len(row)}")
    r = row[0]
    kname = r["Name"].split("(")[0].replace("void ", "")
    durs = _trace_durations(os.path.join(out, "stats"), needle)
    mean = float(r["AverageNs"]) / 1e3
    med = sorted(durs)[len(durs) // 2]
    avg = med  # the launch time used below: the median dispatch (the first ones run while clocks ramp)
    lines = [f"# Fused step, {title} (FP64) — kernel timings", "",
             "Command:", "", "    " + cmd("--kernel-trace --stats", 200), "",
             "| kernel | calls | avg us | median us | min us | max us | % of GPU time |",
             "|---|---|---|---|---|---|---|"]
    for q in sorted(stats, key=lambda q: -float(q["TotalDurationNs"]))[:6]:
        name = q["Name"].split("(")[0].replace("void ", "")
        qd = _trace_durations(os.path.join(out, "stats"), name) or [float("nan")]
        lines.append(f"| `{name[:80]}` | {q['Calls']} | {float(q['AverageNs']) / 1e3:.2f} | "
                     f"{sorted(qd)[len(qd) // 2]:.2f} | {float(q['MinNs']) / 1e3:.2f} | "
                     f"{float(q['MaxNs']) / 1e3:.2f} | {float(q['Percentage']):.1f} |")
    lines += ["", f"Band height {tile_rows} rows.  The {r['Calls']} calls of `{kname}` are the warm-up and "
                  f"the timed steps, one launch per step; the median dispatch takes {med:.2f} us (mean {mean:.2f} us) = "
                  f"{cells / (avg * 1e-6):.3e} cell-updates/s, {alg / (avg * 1e-6) / 1e9:.0f} GB/s of "
                  f"algorithmic traffic ({bench.B_ALG[w['model']]} B per cell-update: the state read and "
                  f"written once), {alg / (avg * 1e-6) / bench.HBM_PEAK * 100:.1f}% of 8 TB/s."]
    with open(os.path.join(PROFILES, f"fwd_{workload}_kernel_stats.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    fetch = _counters(os.path.join(out, "fetch"))
    write = _counters(os.path.join(out, "write"))
    f_k, w_k = _pick(fetch, needle, "FETCH_SIZE"), _pick(write, needle, "WRITE_SIZE")
    f_c, w_c = _pick(fetch, CALIB, "FETCH_SIZE"), _pick(write, CALIB, "WRITE_SIZE")
    fs, wsc = CALIB_BYTES / 1024 / f_c, CALIB_BYTES / 1024 / w_c
    hbm = (f_k * fs + w_k * wsc) * 1024
    sq = _counters(os.path.join(out, "sq"))
    g = {c: _pick(sq, needle, c) for c in SQ_COUNTERS}
    rec = {"kernel": kname, "workload": workload, "cells": cells,
           "kernel_sha": bench.kernel_hash(), "tile_rows": tile_rows,
           "mean_launch_us": mean, "median_launch_us": med,
           "fetch_kib_per_dispatch": round(f_k, 1), "write_kib_per_dispatch": round(w_k, 1),
           "calibration": {"kernel": "torch.add(src, 0.0, out=dst), 2^26 doubles",
                           "bytes_read": CALIB_BYTES, "bytes_written": CALIB_BYTES,
                           "fetch_kib": round(f_c, 1), "write_kib": round(w_c, 1),
                           "fetch_scale": fs, "write_scale": wsc},
           "hbm_bytes_per_launch": hbm, "algorithmic_bytes_per_launch": alg,
           "valu_instructions_per_launch": g["SQ_INSTS_VALU"],
           "lane_instructions_per_cell_update": g["SQ_INSTS_VALU"] * 64 / cells,
           "sq": g}
    with open(bench.counters_file(workload), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    waves = g["SQ_WAVES"]
    lines = [f"# Fused step, {title} — hardware counters", "",
             "Commands (each a run of its own):", "",
             "    " + cmd("--pmc FETCH_SIZE", 200) + " --calibration-copy",
             "    " + cmd("--pmc WRITE_SIZE", 200) + " --calibration-copy",
             "    " + cmd("--pmc " + " ".join(SQ_COUNTERS), 200),
             f"    python3 <repo>/bench_profile.py --forward <out> {workload} {tile_rows}", "",
             "## Memory traffic (KiB per dispatch)", "",
             "| kernel | FETCH_SIZE | WRITE_SIZE |", "|---|---|---|",
             f"| `{kname}` | {f_k:.1f} | {w_k:.1f} |",
             f"| calibration copy, 2^26 doubles (512 MiB in, 512 MiB out) | {f_c:.0f} | {w_c:.0f} |", "",
             f"Calibration: FETCH_SIZE is scaled by {fs:.3f} and WRITE_SIZE by {wsc:.3f}. Scaled traffic per "
             f"launch: {f_k * fs:.0f} KiB read + {w_k * wsc:.0f} KiB written = {hbm / 1e6:.1f} MB, against "
             f"{alg / 1e6:.1f} MB algorithmic ({hbm / alg:.2f}x).", "",
             "## Instruction and occupancy counters (per dispatch)", "",
             "| counter | value | per wave |", "|---|---|---|"]
    for c in SQ_COUNTERS:
        lines.append(f"| {c} | {g[c]:.4g} | {g[c] / waves:.4g} |")
    lines += ["", f"Lane-instructions per cell-update: {g['SQ_INSTS_VALU'] * 64 / cells:.0f}. VALU issue "
                  f"rate at the {avg:.1f} us median launch: "
                  f"{g['SQ_INSTS_VALU'] * 64 / (avg * 1e-6) / bench.VALU_LANE_ISSUE_PEAK * 100:.0f}% of the "
                  f"{bench.VALU_LANE_ISSUE_PEAK / 1e12:.1f} T lane-instructions/s capacity. Share of wave "
                  f"time issuing VALU: {g['SQ_ACTIVE_INST_VALU'] / g['SQ_WAVE_CYCLES']:.2f}; waiting on "
                  f"dependencies (memory): {g['SQ_WAIT_INST_ANY'] / g['SQ_WAVE_CYCLES']:.2f}."]
    with open(os.path.join(PROFILES, f"fwd_{workload}_counters.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps(rec, indent=1))


STAGE3_KINDS = [  # (kernel, template tail, role, arrays read, arrays written), three fields each
    ("stage3d_kernel", "false, false, false, 0>", "stage 1: reads z, writes k1", 1, 1),
    ("stage3d_kernel", "false, true, false, 0>", "stages 2, 3: read z and k_{s-1}, write k_s", 2, 1),
    ("stage3d_kernel", "false, true, true, 0>", "stage 4: reads z, k1, k2, k3, writes z'", 4, 1),
    ("adjoint3d_kernel", "true, false, true, 0>", "adjoint stage 4: reads z, k3, lambda, writes Ybar, zbar", 3, 2),
    ("adjoint3d_kernel", "true, true, true, 0>",
     "adjoint stages 3, 2: read z, k, lambda, Ybar, zbar, write Ybar, zbar", 5, 2),
    ("adjoint3d_kernel", "false, true, false, 0>", "adjoint stage 1: reads z, lambda, Ybar, zbar, writes lambda_n",
     4, 1),
]


def main_3d(out: str) -> None:
    cells = 256 ** 3
    arr = 3 * 8 * cells  # one three-field array
    cmd = lambda extra: (f"cd /tmp && rocprofv3 {extra} --output-format csv -d <out> -o k3 -- "
                         "python3 <repo>/bench.py --only-workload fk_256cube_lap27_rk4")
    stats = _rows(os.path.join(out, "stats"), "*kernel_stats.csv")
    fetch = _counters(os.path.join(out, "fetch"))
    write = _counters(os.path.join(out, "write"))
    with open(os.path.join(PROFILES, "fwd_fk_1024_rk4_counters.json")) as fh:
        cal = json.load(fh)["calibration"]
    fs, wsc = cal["fetch_scale"], cal["write_scale"]
    lines = ["# 3-D RK4 step and adjoint, Fenton-Karma 256^3 (compact 27-point operator, FP64) — stage kernels", "",
             "Commands (each a run of its own), then `python3 <repo>/bench_profile.py --stage3d <out>`:", "",
             "    " + cmd("--kernel-trace --stats"), "    " + cmd("--pmc FETCH_SIZE"), "    " + cmd("--pmc WRITE_SIZE"), "",
             "Algorithmic bytes: the arrays each launch must read and write once (three fields of 8 bytes per "
             "cell each).  HBM bytes: FETCH_SIZE and WRITE_SIZE per dispatch scaled by the factors measured on a "
             f"plain copy (`profiles/fwd_fk_1024_rk4_counters.md`: {fs:.3f} and {wsc:.3f}).", "",
             "| kernel | role | calls | avg us | algorithmic GB/s | of 8 TB/s | HBM bytes / algorithmic |",
             "|---|---|---|---|---|---|---|"]
    per = {}
    for kern, tail, role, nr, nw in STAGE3_KINDS:
        row = [r for r in stats if kern in r["Name"] and r["Name"].split("(")[0].endswith(tail)]
        if not row:
            continue
        r = row[0]
        name = r["Name"].split("(")[0].replace("void ", "")
        avg = float(r["AverageNs"]) / 1e3
        alg = (nr + nw) * arr
        fk = [v for (k, c), v in fetch.items() if k.split("(")[0].replace("void ", "") == name]
        wk = [v for (k, c), v in write.items() if k.split("(")[0].replace("void ", "") == name]
        ratio = (fk[0] * fs + wk[0] * wsc) * 1024 / alg if fk and wk else float("nan")
        per[(kern, tail)] = avg
        lines.append(f"| `{name}` | {role} | {r['Calls']} | {avg:.1f} | {alg / avg / 1e3:.0f} | "
                     f"{alg / avg / 1e3 / 8000 * 100:.0f}% | {ratio:.2f} |")
    fwd = (per[("stage3d_kernel", "false, false, false, 0>")] + 2 * per[("stage3d_kernel", "false, true, false, 0>")]
           + per[("stage3d_kernel", "false, true, true, 0>")])
    lines += ["", f"Forward step (stages 1 + 2 x middle + 4): {fwd:.0f} us = {cells / (fwd * 1e-6):.3e} "
                  f"cell-updates/s.  Against the step's algorithmic traffic, the state read and written once "
                  f"(48 B per cell-update), that is {48 * cells / (fwd * 1e-6) / 8e12 * 100:.1f}% of 8 TB/s; the "
                  f"four stage launches move 312 B per cell-update between them, which they stream at "
                  f"{312 * cells / (fwd * 1e-6) / 8e12 * 100:.0f}% of 8 TB/s.  A plain device-to-device copy "
                  "reaches about 5.3 TB/s (66%) on the same box."]
    with open(os.path.join(PROFILES, "stage3d_fk_256cube_lap27_rk4_kernel_stats.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main_barkley8192(out: str) -> None:
    """Timed-phase launches only: the trace's last 16 dispatches of the
    two-step sweep (the benchmark times two repetitions of 8 launches; the
    earlier dispatches are warm-up and the tuner's trials)."""
    kern = "rd::sweep_kernel<1, 5, 4, 0, 2, 0, 0>"
    cells = 8192 * 8192
    cmd = lambda extra: (f"cd /tmp && rocprofv3 {extra} --output-format csv -d <out> -o bk -- "
                         "python3 <repo>/bench.py --only-workload barkley_8192_rk4_beyond_llc")
    trace = [r for r in _rows(os.path.join(out, "stats"), "*kernel_trace.csv") if kern in r["Kernel_Name"]]
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in trace][-16:]
    avg = sum(durs) / len(durs)

    def last(kind, counter):
        rows = [r for r in _rows(os.path.join(out, kind), "*counter_collection.csv")
                if kern in r["Kernel_Name"] and r["Counter_Name"] == counter]
        vals = [float(r["Counter_Value"]) for r in rows][-16:]
        return sum(vals) / len(vals)
    with open(os.path.join(PROFILES, "fwd_fk_1024_rk4_counters.json")) as fh:
        cal = json.load(fh)["calibration"]
    rd_b = last("fetch", "FETCH_SIZE") * cal["fetch_scale"] * 1024
    wr_b = last("write", "WRITE_SIZE") * cal["write_scale"] * 1024
    state = 2 * 8 * cells
    lines = ["# HBM-bound 2-D probe: Barkley 8192^2 (5-point, RK4, FP64), two steps per launch — kernel timings and traffic", "",
             "Commands (each a run of its own), then `python3 <repo>/bench_profile.py --barkley8192 <out>`:", "",
             "    " + cmd("--kernel-trace --stats"), "    " + cmd("--pmc FETCH_SIZE"), "    " + cmd("--pmc WRITE_SIZE"), "",
             f"Kernel `{kern}`: the fused sweep chaining two RK4 steps per launch.  Timed-phase launches "
             f"(the last 16 dispatches): average {avg:.1f} us (min {min(durs):.1f}, max {max(durs):.1f}).", "",
             "| quantity | per launch (two steps) |", "|---|---|",
             f"| state read + written once (algorithmic for the launch) | {2 * state / 1e9:.3f} GB |",
             f"| single-step algorithmic bytes x 2 steps (32 B per cell-update) | {4 * state / 1e9:.3f} GB |",
             f"| HBM read (FETCH_SIZE x {cal['fetch_scale']:.3f}) | {rd_b / 1e9:.3f} GB |",
             f"| HBM written (WRITE_SIZE x {cal['write_scale']:.3f}) | {wr_b / 1e9:.3f} GB |", "",
             f"Rate: {2 * cells / (avg * 1e-6):.3e} cell-updates/s; single-step algorithmic bandwidth "
             f"{4 * state / (avg * 1e-6) / 1e12:.2f} TB/s ({4 * state / (avg * 1e-6) / 8e12 * 100:.0f}% of 8 TB/s); "
             f"measured HBM traffic {(rd_b + wr_b) / (avg * 1e-6) / 1e12:.2f} TB/s "
             f"({(rd_b + wr_b) / (2 * state):.2f}x the launch's algorithmic bytes: halo columns and band "
             "ramps re-read).  Calibration factors from `profiles/fwd_fk_1024_rk4_counters.md`."]
    with open(os.path.join(PROFILES, "fwd_barkley_8192_rk4_kernel_stats.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


TANGENT_KERNEL = "rd::sweep_kernel<2, 9, 4, 1, 1, 0, 1>"


def main_tangent(out: str, tile_rows: int) -> None:
    """The exact tangent step (rd_jvp) of the same workload: OUT/stats with
    the kernel trace, OUT/fetch and OUT/write with the counters, each a run of
    `bench.py` at the tangent's band height (which fixes the forward's too)."""
    cells = 1024 * 1024
    alg = 4 * 3 * 8 * cells  # read and write the state and its tangent once
    cmd = lambda extra: (f"cd /tmp && rocprofv3 {extra} --output-format csv -d <out> -o tan -- "
                         f"python3 <repo>/bench.py --steps 200 --warmup 2 --no-cpu-baseline --no-other-workloads "
                         f"--variant sweep --tile-rows {tile_rows}")
    stats = _rows(os.path.join(out, "stats"), "*kernel_stats.csv")
    row = [r for r in stats if r["Name"].startswith("void " + TANGENT_KERNEL)]
    if not row:
        raise RuntimeError("no tangent kernel in the trace")
    r = row[0]
    # the first launches run while the clocks ramp up: use the median dispatch
    trace = [t for t in _rows(os.path.join(out, "stats"), "*kernel_trace.csv")
             if t["Kernel_Name"].startswith("void " + TANGENT_KERNEL)]
    durs = sorted((int(t["End_Timestamp"]) - int(t["Start_Timestamp"])) / 1e3 for t in trace)
    avg = durs[len(durs) // 2]
    fetch = _counters(os.path.join(out, "fetch"))
    write = _counters(os.path.join(out, "write"))
    f_k, w_k = _pick(fetch, TANGENT_KERNEL, "FETCH_SIZE"), _pick(write, TANGENT_KERNEL, "WRITE_SIZE")
    with open(os.path.join(PROFILES, "fwd_fk_1024_rk4_counters.json")) as fh:
        cal = json.load(fh)["calibration"]
    fs, wsc = cal["fetch_scale"], cal["write_scale"]
    hbm = (f_k * fs + w_k * wsc) * 1024
    lines = ["# Exact tangent step (rd_jvp), Fenton-Karma 1024x1024 (9-point, RK4, FP64)", "",
             "Commands (each a run of its own), then `python3 <repo>/bench_profile.py --tangent <out> "
             f"{tile_rows}`:", "",
             "    " + cmd("--kernel-trace --stats"), "    " + cmd("--pmc FETCH_SIZE"), "    " + cmd("--pmc WRITE_SIZE"),
             "", f"Band height {tile_rows} rows (the autotuner's choice for the tangent on this grid).", "",
             "| kernel | calls | median us | mean us | min us | max us | algorithmic GB/s (median) | of 8 TB/s | "
             "HBM bytes / algorithmic |",
             "|---|---|---|---|---|---|---|---|---|",
             f"| `{TANGENT_KERNEL}` | {r['Calls']} | {avg:.2f} | {float(r['AverageNs']) / 1e3:.2f} | "
             f"{float(r['MinNs']) / 1e3:.2f} | "
             f"{float(r['MaxNs']) / 1e3:.2f} | {alg / avg / 1e3:.0f} | {alg / avg / 1e3 / 8000 * 100:.0f}% | "
             f"{hbm / alg:.2f} |", "",
             f"Algorithmic bytes per launch: {alg / 1e6:.1f} MB (96 per cell-update: the three fields and their "
             f"tangents read and written once). Counters per dispatch: FETCH_SIZE {f_k:.0f} KiB, WRITE_SIZE "
             f"{w_k:.0f} KiB, scaled by {fs:.3f} and {wsc:.3f} (the plain-copy calibration of "
             f"`profiles/fwd_fk_1024_rk4_counters.md`): {hbm / 1e6:.1f} MB. The step runs at "
             f"{cells / (avg * 1e-6):.3e} tangent cell-updates/s."]
    with open(os.path.join(PROFILES, "tan_fk_1024_rk4_kernel_stats.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _calibration(out: str):
    """FETCH_SIZE and WRITE_SIZE scale factors from the plain copy of the
    headline's counter runs (OUT/fetch and OUT/write hold it)."""
    fetch = _counters(os.path.join(out, "fetch"))
    write = _counters(os.path.join(out, "write"))
    f_c, w_c = _pick(fetch, CALIB, "FETCH_SIZE"), _pick(write, CALIB, "WRITE_SIZE")
    return CALIB_BYTES / 1024 / f_c, CALIB_BYTES / 1024 / w_c


def _kernel_table(out: str, kinds, cal_dir: str, title: str, cmd, cells: int = 0):
    """Per-kernel timing (median dispatch) and counter traffic against the
    algorithmic bytes each launch must move.  kinds: (name prefix, role,
    algorithmic bytes per launch).  With OUT/sq (a run counting SQ_WAVES and
    SQ_INSTS_VALU) and the cells one launch updates, also the VALU
    lane-instructions per cell and launch and the share of the VALU issue
    capacity at the median dispatch."""
    fs, wsc = _calibration(cal_dir)
    fetch = _counters(os.path.join(out, "fetch"))
    write = _counters(os.path.join(out, "write"))
    sq = _counters(os.path.join(out, "sq")) if cells and os.path.isdir(os.path.join(out, "sq")) else None
    stats = _rows(os.path.join(out, "stats"), "*kernel_stats.csv")
    head = "| kernel | role | calls | median us | algorithmic MB | algorithmic GB/s | of 8 TB/s | HBM MB | HBM / algorithmic |"
    rule = "|---|---|---|---|---|---|---|---|---|"
    cmds = ["    " + cmd("--kernel-trace --stats"), "    " + cmd("--pmc FETCH_SIZE"), "    " + cmd("--pmc WRITE_SIZE")]
    if sq is not None:
        head += " VALU lane-instr per cell | VALU issue |"
        rule += "---|---|"
        cmds.append("    " + cmd("--pmc SQ_WAVES SQ_INSTS_VALU"))
    lines = [f"# {title}", "", "Commands (each a run of its own):", "", *cmds,
             "", f"HBM bytes: FETCH_SIZE x {fs:.3f} + WRITE_SIZE x {wsc:.3f} per dispatch (the factors a plain copy of "
             "2^26 doubles reads in the headline's counter runs).", "", head, rule]
    med = {}
    for needle, role, alg in kinds:
        row = [r for r in stats if r["Name"].startswith("void " + needle)]
        if len(row) != 1:
            raise RuntimeError(f"expected one kernel {needle!r}, found {len(row)}")
        durs = sorted(_trace_durations(os.path.join(out, "stats"), "void " + needle))
        m = durs[len(durs) // 2]
        med[needle] = m
        f_k, w_k = _pick(fetch, needle, "FETCH_SIZE"), _pick(write, needle, "WRITE_SIZE")
        hbm = (f_k * fs + w_k * wsc) * 1024
        line = (f"| `{needle}` | {role} | {row[0]['Calls']} | {m:.2f} | {alg / 1e6:.1f} | {alg / m / 1e3:.0f} | "
                f"{alg / m / 1e3 / 8000 * 100:.0f}% | {hbm / 1e6:.1f} | {hbm / alg:.2f} |")
        if sq is not None:
            lanes = _pick(sq, needle, "SQ_INSTS_VALU") * 64
            line += f" {lanes / cells:.0f} | {lanes / (m * 1e-6) / bench.VALU_LANE_ISSUE_PEAK * 100:.0f}% |"
        lines.append(line)
    return med, lines


def _write(fname: str, lines) -> None:
    with open(os.path.join(PROFILES, fname), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main_ensemble(out: str, cal_dir: str) -> None:
    """The 64-member Fenton-Karma ensemble (16 each of 256^2 .. 768^2, RK4):
    the batched forward and tangent kernels, from three runs of
    `bench.py --only-workload fk_ensemble_64_jvp`."""
    import rd_inputs as ri
    cells = sum(w["nx"] * w["ny"] for w in ri.fk_batch_workloads(nsteps=1))
    cmd = lambda extra: (f"cd /tmp && rocprofv3 {extra} --output-format csv -d <out> -o p -- "
                         "python3 <repo>/bench.py --only-workload fk_ensemble_64_jvp")
    fwd, tan = "rd::batch_sweep_kernel<2, 9, 4, 0, 0, 1>", "rd::batch_sweep_kernel<2, 9, 4, 1, 0, 1>"
    med, lines = _kernel_table(out, [(fwd, "one RK4 step of all 64 members", 48 * cells),
                                     (tan, "one RK4 step of all members and their tangents", 96 * cells)],
                               cal_dir, "Batched ensemble, 64 Fenton-Karma members (9-point, RK4, FP64) — one launch "
                               "per step", cmd, cells)
    lines += ["", f"{cells} cells per launch (16 each of 256^2, 384^2, 512^2, 768^2).  Algorithmic bytes: the state "
                  "(48 B per cell) or the state and tangent (96 B) read and written once.  The tangent step costs "
                  f"{med[tan] / med[fwd]:.2f}x the forward step."]
    _write("ens_fk_64_members_rk4_kernel_stats.md", lines)


def main_adjoint(out: str, cal_dir: str) -> None:
    """The adjoint workload (Barkley 1024^2, 5-point, RK4, 4000 steps,
    checkpoints every 64): forward with checkpoints, then per reverse step the
    segment recompute and either the fused reverse step (stage inputs
    recomputed inside it) or the stage-input sweep and the adjoint kernel,
    from three runs of `bench.py --only-workload barkley_1024_rk4_adjoint_4000`."""
    cells = 1024 * 1024
    field = 8 * cells
    cmd = lambda extra: (f"cd /tmp && rocprofv3 {extra} --output-format csv -d <out> -o p -- "
                         "python3 <repo>/bench.py --only-workload barkley_1024_rk4_adjoint_4000")
    fused = "rd::adjoint_fused_kernel<1, 5, 4>"
    adj, stg = "rd::adjoint_kernel<1, 5, 4, 0>", "rd::sweep_kernel<1, 5, 4, 2, 1, 0, 0>"
    rec1, fwd2 = "rd::sweep_kernel<1, 5, 4, 0, 1, 0, 0>", "rd::sweep_kernel<1, 5, 4, 0, 2, 0, 0>"
    stats = _rows(os.path.join(out, "stats"), "*kernel_stats.csv")
    has = lambda needle, n=100: any(r["Name"].startswith("void " + needle) and int(r["Calls"]) > n for r in stats)
    kinds = [(rec1, "forward step, one per launch (state read and written once)", 4 * field)]
    if has(fwd2):
        kinds.insert(0, (fwd2, "forward, two steps per launch (state read and written once)", 4 * field))
    if has(fused):
        kinds.append((fused, "one reverse step, stage inputs recomputed (reads z and lambda; writes lambda)",
                      6 * field))
    else:
        kinds += [(stg, "stage inputs Y2..Y4 of one step (reads z, writes three states)", 8 * field),
                  (adj, "one reverse step (reads z, Y2..Y4, lambda; writes lambda)", 12 * field)]
    med, lines = _kernel_table(out, kinds, cal_dir, "Adjoint workload, Barkley 1024x1024 (5-point, RK4, FP64) — "
                               "forward and reverse kernels", cmd, cells)
    fwd_step = med[fwd2] / 2 if fwd2 in med else med[rec1]
    if fused in med:
        rev = med[fused] + med[rec1]
        tail = "32 (recompute) + 48 (fused reverse step) = 80, 2.5 times the forward's 32."
        what = "segment recompute + fused reverse step"
    else:
        rev = med[adj] + med[stg] + med[rec1]
        tail = "32 (recompute) + 64 (stage inputs) + 96 (adjoint) = 192, six times the forward's 32."
        what = "segment recompute + stage inputs + adjoint"
    lines += ["", f"Per reverse step: {what} = {rev:.1f} us, {rev / fwd_step:.2f}x the forward step "
                  f"({fwd_step:.2f} us).  Bytes per cell and reverse step: {tail}"]
    _write("adj_barkley_1024_rk4_kernel_stats.md", lines)


def main_headline(out: str) -> None:
    """Kernel timings of the benchmark's own headline command (default steps,
    warm-up and timing windows, the band height of the committed counter
    record), to set beside the launch time bench.py measures with events:
    `rocprofv3 --kernel-trace --stats ... -- python3 bench.py --no-cpu-baseline
    --no-jvp --no-other-workloads` into OUT."""
    import rd_inputs as ri
    w = ri.workload(bench.HEADLINE)
    needle = sweep_kernel(w)
    stats = _rows(out, "*kernel_stats.csv")
    row = [r for r in stats if needle in r["Name"]]
    if len(row) != 1:
        raise RuntimeError(f"expected one kernel matching {needle!r}, found {len(row)}")
    r = row[0]
    durs = _trace_durations(out, needle)
    med = sorted(durs)[len(durs) // 2]
    cells = w["nx"] * w["ny"]
    alg = bench.B_ALG[w["model"]] * cells
    kname = r["Name"].split("(")[0].replace("void ", "")
    lines = [f"# Headline benchmark command under the profiler: {w['model']} {w['nx']}x{w['ny']}, {w['stencil']}, "
             f"{w['scheme']} (FP64)", "", "Command:", "",
             "    cd /tmp && rocprofv3 --kernel-trace --stats --output-format csv -d <out> -o p -- python3 "
             "<repo>/bench.py --no-cpu-baseline --no-jvp --no-other-workloads",
             f"    python3 <repo>/bench_profile.py --headline <out>", "",
             "| kernel | calls | average us | median us | min us | max us |", "|---|---|---|---|---|---|",
             f"| `{kname}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | {med:.2f} | "
             f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |", "",
             f"The calls are the warm-up and the five timed windows of 200 steps (one launch per step) at the band "
             f"height of the committed counter record.  Average {float(r['AverageNs']) / 1e3:.2f} us = "
             f"{alg / (float(r['AverageNs']) * 1e-9) / 1e9:.0f} GB/s of algorithmic traffic "
             f"({alg / (float(r['AverageNs']) * 1e-9) / bench.HBM_PEAK * 100:.1f}% of 8 TB/s); bench.py's event-timed "
             "launch time in the same run is printed in its JSON line (`roofline.avg_launch_us`)."]
    with open(os.path.join(PROFILES, f"fwd_{bench.HEADLINE}_bench_command_stats.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1] == "--barkley8192":
        main_barkley8192(sys.argv[2])
    elif sys.argv[1] == "--stage3d":
        main_3d(sys.argv[2])
    elif sys.argv[1] == "--tangent":
        main_tangent(sys.argv[2], int(sys.argv[3]))
    elif sys.argv[1] == "--forward":
        main_forward(sys.argv[2], sys.argv[3], int(sys.argv[4]))
    elif sys.argv[1] == "--headline":
        main_headline(sys.argv[2])
    elif sys.argv[1] == "--ensemble":
        main_ensemble(sys.argv[2], sys.argv[3])
    elif sys.argv[1] == "--adjoint":
        main_adjoint(sys.argv[2], sys.argv[3])
    else:
        raise SystemExit(__doc__)
