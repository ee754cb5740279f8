"""rd_step_batched: many problems on uneven grids in one launch per step must
equal per-problem rd_step / rd_jvp bit for bit (and hence the oracle)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import paper_1309_1720_amd as rd
import rd_inputs as ri
from rdtest import dev, host, problems, rel_linf

pytestmark = pytest.mark.gpu

SIZES = [(40, 40), (64, 64), (97, 61), (130, 70), (1, 5), (57, 1), (200, 33)]


def batch_setup(model, stencil, scheme, steps, sizes=SIZES, seed=0):
    base = {"barkley": "barkley_1024_rk4_adjoint", "fk": "fk_1024_rk4", "bocf": "bocf_2048_aniso_rk4",
            "fhn": "fhn_256_rk4",
            "diffusion": "bocf_2048_aniso_rk4"}[model]
    out = []
    for k, (nx, ny) in enumerate(sizes):
        w = ri.workload(base, model=model, stencil=stencil, scheme=scheme, nx=nx, ny=ny)
        po, pr = problems(w, nsteps=steps)
        z0 = ri.random_fields(model, nx, ny, seed + k)
        v = ri.direction(len(z0), nx, ny, seed + 100 + k)
        out.append((po, pr, z0, v))
    return out


@pytest.mark.parametrize("model,stencil,scheme", [("fk", "lap9", "rk4"), ("barkley", "lap5", "euler"),
                                                  ("fhn", "lap9_aniso", "rk4"), ("bocf", "lap9", "rush_larsen"),
                                                  ("fk", "lap5", "implicit_euler"),
                                                  ("bocf", "lap9_aniso", "heun"), ("diffusion", "lap9", "rk4")])
@pytest.mark.parametrize("steps", [1, 6])
@pytest.mark.parametrize("tangent", [False, True])
def test_batched_equals_single_bitwise(model, stencil, scheme, steps, tangent):
    cases = batch_setup(model, stencil, scheme, steps)
    fields = [dev(z0) for _, _, z0, _ in cases]
    tans = [dev(v) for _, _, _, v in cases] if tangent else None
    rd.step_batched([pr for _, pr, _, _ in cases], fields, tans)
    for k, (po, pr, z0, v) in enumerate(cases):
        zs, vs = dev(z0), dev(v)
        if tangent:
            rd.jvp(pr, zs, vs)
        else:
            rd.step(pr, zs)
        assert all(np.array_equal(a, b) for a, b in zip(host(fields[k]), host(zs))), k
        if tangent:
            assert all(np.array_equal(a, b) for a, b in zip(host(tans[k]), host(vs))), k


def test_batched_tangent_matches_oracle():
    cases = batch_setup("fk", "lap9", "rk4", 25, sizes=[(48, 48), (72, 72), (96, 96)], seed=4000)
    fields = [dev(z0) for _, _, z0, _ in cases]
    tans = [dev(v) for _, _, _, v in cases]
    rd.step_batched([pr for _, pr, _, _ in cases], fields, tans)
    for k, (po, pr, z0, v) in enumerate(cases):
        zr, jr = oracle.jvp(po, z0, v, 25)
        assert rel_linf(host(fields[k]), zr) <= 1e-11
        assert rel_linf(host(tans[k]), jr) <= 1e-11


@pytest.mark.parametrize("field,value", [("dx", 0.03), ("nsteps", 3), ("step_k", 20.0)])
def test_batched_rejects_mixed_physics(field, value):
    cases = batch_setup("fk", "lap9", "rk4", 2, sizes=[(16, 16), (20, 20)])
    probs = [pr for _, pr, _, _ in cases]
    setattr(probs[1], field, value)
    with pytest.raises(rd.RDError, match="RD_EUNSUPPORTED"):
        rd.step_batched(probs, [dev(z0) for _, _, z0, _ in cases])


@pytest.mark.parametrize("model,stencil,scheme", [("barkley", "lap5", "rk4"), ("fk", "lap9", "rk4"),
                                                  ("bocf", "lap9_aniso", "rush_larsen")])
@pytest.mark.parametrize("tangent", [False, True])
def test_batched_time_steps_per_instance(model, stencil, scheme, tangent):
    """Members with different time steps (periodic orbits of different
    periods at a common step count) in one batched call: each equals its own
    single call bit for bit."""
    cases = batch_setup(model, stencil, scheme, 5, sizes=[(40, 36), (64, 50), (33, 70)])
    probs = [pr for _, pr, _, _ in cases]
    for k, pr in enumerate(probs):
        pr.dt = pr.dt * (1.0 - 0.125 * k)
    fields = [dev(z0) for _, _, z0, _ in cases]
    tans = [dev(v) for _, _, _, v in cases] if tangent else None
    rd.step_batched(probs, fields, tans)
    for k, ((po, _, z0, v), pr) in enumerate(zip(cases, probs)):
        zs, vs = dev(z0), dev(v)
        if tangent:
            rd.jvp(pr, zs, vs)
        else:
            rd.step(pr, zs)
        assert all(np.array_equal(a, b) for a, b in zip(host(fields[k]), host(zs))), k
        if tangent:
            assert all(np.array_equal(a, b) for a, b in zip(host(tans[k]), host(vs))), k
    if not tangent:
        # and against the oracle at that member's own step
        po = dataclasses.replace(cases[-1][0], dt=probs[-1].dt)
        ref = oracle.step(po, cases[-1][2], 5)
        assert rel_linf(host(fields[-1]), ref) <= 1e-11


def test_ensemble_workload_shapes_one_step():
    """The 64-instance ensemble (16 each of 256^2, 384^2, 512^2, 768^2) with
    tangents, one step, against per-instance calls on a sample of members."""
    ws = ri.fk_batch_workloads(nsteps=1)
    params = ri.params_array("fk")
    probs = [rd.Problem.from_workload(w, params) for w in ws]
    z0s = [ri.fk_ic(w["nx"], w["ny"], w["seed"]) for w in ws]
    vs = [ri.direction(3, w["nx"], w["ny"], w["direction_seed"]) for w in ws]
    fields = [dev(z) for z in z0s]
    tans = [dev(v) for v in vs]
    rd.step_batched(probs, fields, tans)
    for k in (0, 17, 40, 63):
        zs, vt = dev(z0s[k]), dev(vs[k])
        rd.jvp(probs[k], zs, vt)
        assert all(np.array_equal(a, b) for a, b in zip(host(fields[k]), host(zs)))
        assert all(np.array_equal(a, b) for a, b in zip(host(tans[k]), host(vt)))
