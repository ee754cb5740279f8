"""GPU parity at the workloads' full sizes and horizons, in the launch
configuration the benchmark times (autotuned plans, one fused launch per
step, the batched ensemble call), against the oracle's results stored by
tests/golden/make_fullsize_goldens.py (sampled cells: corner, edge and centre
windows, the middle row and column, seeded random cells; the relative
L-infinity error divides by the oracle's whole-grid maximum of each field).
"""
import os
import sys

import numpy as np
import pytest
import torch

import paper_1309_1720_amd as rd
import rd_inputs as ri
from rdtest import dev, host, problems

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_fullsize_goldens as golden  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-11  # relative L-infinity, per field


def check_sample(got, g, key="state", what=""):
    """Element-wise comparison of full-grid device results with a stored sample."""
    iy, ix = g["iy"], g["ix"]
    ref, scale = g[key], g[f"{key}_max"]
    worst = 0.0
    for f, a in enumerate(got):
        vals = a[iy, ix]
        assert np.isfinite(vals).all(), (what, key, f)
        err = float(np.max(np.abs(vals - ref[f]))) / float(scale[f])
        worst = max(worst, err)
        # the sample's own maximum is a lower bound of the whole-grid one
        assert float(np.max(np.abs(a))) >= float(np.max(np.abs(ref[f])))
    print(f"{what} {key}: rel-Linf over {len(iy)} sampled cells {worst:.3e}")
    assert worst <= TOL, (what, key, worst)
    return worst


def test_fk_1024_thousand_steps():
    """Fenton-Karma 1024^2, 9-point, RK4: 1000 steps of the whole grid."""
    g = golden.load("fk_1024_rk4", 1000)
    w = ri.workload("fk_1024_rk4")
    _, pr = problems(w, nsteps=1000)
    zt = dev(ri.initial_condition(w))
    rd.step(pr, zt)
    check_sample(host(zt), g, what="fk 1024^2 1000 steps")


@pytest.mark.parametrize("horizon", [200, 1000])
def test_bocf_2048_full_grid(horizon):
    """Bueno-Orovio 2048^2, anisotropic flux form, RK4: the whole grid after
    200 and after 1000 steps."""
    g = golden.load("bocf_2048_aniso_rk4", horizon)
    w = ri.workload("bocf_2048_aniso_rk4")
    _, pr = problems(w, nsteps=horizon)
    zt = dev(ri.initial_condition(w))
    rd.step(pr, zt)
    check_sample(host(zt), g, what=f"bocf 2048^2 {horizon} steps")


def test_ensemble_jvp_one_member_per_size_two_hundred_steps():
    """The 64-member Fenton-Karma ensemble (16 each of 256^2 .. 768^2) with
    its seeded unit directions, advanced 200 RK4 steps with tangents in the
    batched call; the first member of each size against the oracle's state
    and complex-step JVP."""
    members = ri.fk_batch_workloads(nsteps=200)
    params = ri.params_array("fk")
    probs = [rd.Problem.from_workload(m, params) for m in members]
    fields = [dev(ri.initial_condition(m)) for m in members]
    tans = [dev(ri.direction(3, m["nx"], m["ny"], m["direction_seed"])) for m in members]
    rd.step_batched(probs, fields, tans)
    torch.cuda.synchronize()
    for n in ri.FK_BATCH_SIZES:
        i = next(k for k, m in enumerate(members) if m["nx"] == n)
        g = golden.load(f"fk_ensemble_jvp_{n}", 200)
        assert g["meta"]["seed"] == members[i]["seed"]
        assert g["meta"]["direction_seed"] == members[i]["direction_seed"]
        check_sample(host(fields[i]), g, "state", what=f"ensemble {n}^2")
        check_sample(host(tans[i]), g, "tangent", what=f"ensemble {n}^2")
