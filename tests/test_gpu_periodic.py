"""Periodic boundaries (RD_BC_PERIODIC, the alternative to no-flux named in
Sect. 3): GPU parity of the step, the tangent and the adjoint against the
oracle, and properties that hold at any size (translation equivariance, the
Fourier eigenmode of the discrete Laplacian, conservation)."""
import itertools
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1309_1720_amd as rd
import rd_inputs as ri
from rdtest import dev, gpu_step, host, problems, rel_linf

pytestmark = pytest.mark.gpu

TOL = 1e-11
BASE = {"diffusion": "bocf_2048_aniso_rk4", "barkley": "barkley_1024_rk4_adjoint",
        "fk": "fk_1024_rk4", "bocf": "bocf_2048_aniso_rk4", "fhn": "fhn_256_rk4"}
MODELS = ["diffusion", "barkley", "fk", "bocf", "fhn"]
STENCILS = ["lap5", "lap9", "lap9_aniso"]


def setup(model, stencil, scheme, nx, ny, steps, seed=3, **kw):
    w = ri.workload(BASE[model], model=model, stencil=stencil, scheme=scheme, nx=nx, ny=ny,
                    bc="periodic", **kw)
    po, pr = problems(w, nsteps=steps)
    if model == "barkley":
        z0 = ri.barkley_ic(nx, ny, seed)
    elif model == "diffusion":
        z0 = ri.diffusion_ic(nx, ny, seed)
    else:
        z0 = ri.random_fields(model, nx, ny, seed)
    return po, pr, z0


@pytest.fixture
def variant(request):
    rd.set_kernel_variant(request.param)
    yield request.param
    rd.set_kernel_variant(None)


@pytest.mark.parametrize("variant", ["sweep", "pipe"], indirect=True)
@pytest.mark.parametrize("model,stencil,scheme", list(itertools.product(MODELS, STENCILS, ["euler", "heun", "rk4"])))
def test_periodic_step_matches_oracle(model, stencil, scheme, variant):
    """131 x 77 (a ragged strip in x, several bands in y), 23 steps.  The
    pipelined variant does not handle periodic rows; asking for it must still
    give the right answer."""
    po, pr, z0 = setup(model, stencil, scheme, 131, 77, 23)
    ref = oracle.step(po, z0, 23)
    got = gpu_step(pr, z0)
    err = rel_linf(got, ref)
    print(f"periodic {variant} {model} {stencil} {scheme}: rel-Linf {err:.3e}")
    assert err <= TOL
    if model in ("diffusion", "barkley", "fhn") and stencil == "lap5":
        assert all(np.array_equal(g, r) for g, r in zip(got, ref))


@pytest.mark.parametrize("model,stencil,scheme", list(itertools.product(["fk", "bocf"], STENCILS,
                                                                         ["rush_larsen", "implicit_euler"])))
def test_periodic_gate_schemes_match_oracle(model, stencil, scheme):
    po, pr, z0 = setup(model, stencil, scheme, 131, 77, 23)
    ref = oracle.step(po, z0, 23)
    assert rel_linf(gpu_step(pr, z0), ref) <= TOL


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 9), (9, 1), (2, 2), (3, 130), (130, 3), (57, 5), (64, 64), (65, 3)])
@pytest.mark.parametrize("model,stencil,scheme", [("fk", "lap9", "rk4"), ("barkley", "lap5", "heun"),
                                                  ("bocf", "lap9_aniso", "rk4"), ("fhn", "lap9_aniso", "euler")])
def test_periodic_degenerate_and_ragged_grids(nx, ny, model, stencil, scheme):
    """Grids narrower than the halo wrap onto themselves several times."""
    po, pr, z0 = setup(model, stencil, scheme, nx, ny, 6)
    ref = oracle.step(po, z0, 6)
    assert rel_linf(gpu_step(pr, z0), ref) <= TOL


@pytest.mark.parametrize("model,stencil,scheme", [("barkley", "lap5", "euler"), ("barkley", "lap9", "heun"),
                                                  ("diffusion", "lap9_aniso", "euler"), ("fhn", "lap9", "rk4")])
@pytest.mark.parametrize("nx,ny", [(150, 77), (5, 3), (49, 200)])
def test_periodic_steps_per_launch_agree_bitwise(model, stencil, scheme, nx, ny):
    po, pr, z0 = setup(model, stencil, scheme, nx, ny, 17)
    outs = []
    kmax = 8 // {"euler": 1, "heun": 2, "rk4": 4}[scheme]
    try:
        for k in sorted({1, 2, kmax}):
            rd.set_steps_per_launch(k)
            outs.append(gpu_step(pr, z0))
    finally:
        rd.set_steps_per_launch(0)
    for o in outs[1:]:
        assert all(np.array_equal(a, b) for a, b in zip(o, outs[0]))
    assert rel_linf(outs[0], oracle.step(po, z0, 17)) <= TOL


@pytest.mark.parametrize("model,stencil", [("fk", "lap9"), ("barkley", "lap5"), ("fhn", "lap9"),
                                           ("bocf", "lap9_aniso")])
def test_periodic_translation_equivariance_bitwise(model, stencil):
    """Stepping a translated state gives the translated result, bit for bit
    (every cell does the same operations on the same values).  The fibre
    angle varies along x, so the anisotropic operator is only shifted in y."""
    nx, ny = 193, 150
    _, pr, z0 = setup(model, stencil, "rk4", nx, ny, 9)
    a = gpu_step(pr, z0)
    shifts = [(37, 0), (0, 101), (-70, 64)] if stencil != "lap9_aniso" else [(37, 0), (-101, 0)]
    for sy, sx in shifts:
        b = gpu_step(pr, [np.roll(x, (sy, sx), axis=(0, 1)) for x in z0])
        for x, y in zip(a, b):
            assert np.array_equal(np.roll(x, (sy, sx), axis=(0, 1)), y), (sy, sx)


def test_periodic_reflection_bitwise():
    _, pr, z0 = setup("fk", "lap9", "rk4", 97, 66, 8)
    a = gpu_step(pr, z0)
    b = gpu_step(pr, [x[:, ::-1] for x in z0])
    for x, y in zip(a, b):
        assert np.array_equal(x[:, ::-1], y)


@pytest.mark.parametrize("stencil", ["lap5", "lap9"])
def test_periodic_fourier_mode_at_full_size(stencil):
    """On a periodic 1024 x 1024 grid a Fourier mode is an eigenvector of the
    discrete Laplacian: lap5 has eigenvalue -(4/h^2)(sin^2(a/2) + sin^2(b/2)),
    lap9 -(2/(3h^2))(5 - 2cos a - 2cos b - cos a cos b), a = 2 pi kx / nx,
    b = 2 pi ky / ny.  Pure diffusion by explicit Euler multiplies it by
    (1 + dt D lambda) per step.  Checked at the largest grid of the step
    workloads, independent of the oracle."""
    n, steps = 1024, 50
    w = ri.workload("fk_1024_rk4", model="diffusion", stencil=stencil, scheme="euler", nx=n, ny=n, bc="periodic")
    _, pr = problems(w, nsteps=steps)
    kx, ky = 3, 5
    x = np.arange(n)
    mode = np.cos(2 * np.pi * ky * x[:, None] / n + 0.7) * np.cos(2 * np.pi * kx * x[None, :] / n + 0.3)
    a, b = 2 * np.pi * kx / n, 2 * np.pi * ky / n
    h2 = pr.dx ** 2
    if stencil == "lap5":
        lam = -(4.0 / h2) * (math.sin(a / 2) ** 2 + math.sin(b / 2) ** 2)
    else:
        lam = -(2.0 / (3.0 * h2)) * (5 - 2 * math.cos(a) - 2 * math.cos(b) - math.cos(a) * math.cos(b))
    got = gpu_step(pr, [mode])[0]
    expect = (1.0 + pr.dt * pr.D_par * lam) ** steps * mode
    assert np.max(np.abs(got - expect)) <= 1e-12


def test_periodic_aniso_diffusion_conserves_at_full_size():
    """The flux form telescopes on a periodic grid: the total is conserved."""
    w = ri.workload("bocf_2048_aniso_rk4", model="diffusion", stencil="lap9_aniso", scheme="rk4", bc="periodic")
    _, pr = problems(w, nsteps=20)
    z0 = ri.diffusion_ic(w["nx"], w["ny"], 4)
    got = gpu_step(pr, z0)[0]
    assert abs(got.sum() - z0[0].sum()) <= 1e-12 * abs(z0[0]).sum()


def gpu_jvp(pr, z0, v):
    zt, vt = dev(z0), dev(v)
    rd.jvp(pr, zt, vt)
    return host(zt), host(vt)


@pytest.mark.parametrize("model,stencil,scheme", [(m, st, "rk4") for m in MODELS for st in STENCILS]
                         + [("fk", "lap9_aniso", "rush_larsen"), ("bocf", "lap5", "implicit_euler"),
                            ("barkley", "lap9", "heun"), ("fhn", "lap5", "euler")])
def test_periodic_jvp_matches_oracle(model, stencil, scheme):
    po, pr, z0 = setup(model, stencil, scheme, 97, 61, 13)
    v = ri.direction(len(z0), 97, 61, 103)
    z_ref, jv_ref = oracle.jvp(po, z0, v, 13)
    z_gpu, jv_gpu = gpu_jvp(pr, z0, v)
    err = rel_linf(jv_gpu, jv_ref)
    print(f"periodic {model} {stencil} {scheme}: tangent rel-Linf {err:.3e}")
    assert err <= TOL
    assert all(np.array_equal(a, b) for a, b in zip(z_gpu, gpu_step(pr, z0)))


def gpu_vjp(pr, z0, lam):
    zt = dev(z0)
    ck = torch.zeros(max(rd.checkpoint_count(pr), 1) * pr.nfields * pr.nx * pr.ny,
                     dtype=torch.float64, device="cuda")
    rd.step(pr, zt, ck)
    lt = dev(lam)
    rd.vjp(pr, ck, lt)
    return host(lt)


@pytest.mark.parametrize("model,stencil,scheme", [(m, st, sc) for m in MODELS for st in STENCILS
                                                  for sc in ("euler", "rk4")])
def test_periodic_vjp_matches_oracle(model, stencil, scheme):
    po, pr, z0 = setup(model, stencil, scheme, 97, 61, 11, checkpoint_every=4)
    lam = ri.direction(len(z0), 97, 61, 77)
    ref = oracle.vjp(po, z0, lam, 11, checkpoint_every=4)
    err = rel_linf(gpu_vjp(pr, z0, lam), ref)
    print(f"periodic {model} {stencil} {scheme}: adjoint rel-Linf {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 9), (9, 2), (65, 3), (3, 70)])
@pytest.mark.parametrize("stencil", STENCILS)
def test_periodic_vjp_degenerate_grids(nx, ny, stencil):
    po, pr, z0 = setup("fk", stencil, "rk4", nx, ny, 5, checkpoint_every=2)
    lam = ri.direction(len(z0), nx, ny, 9)
    ref = oracle.vjp(po, z0, lam, 5, checkpoint_every=2)
    assert rel_linf(gpu_vjp(pr, z0, lam), ref) <= TOL


@pytest.mark.parametrize("model,stencil", [("bocf", "lap9_aniso"), ("fhn", "lap9"), ("barkley", "lap5")])
def test_periodic_dot_product(model, stencil):
    """<lambda, J v> = <J^T lambda, v> for the GPU tangent and adjoint."""
    nx, ny = 140, 90
    _, pr, z0 = setup(model, stencil, "rk4", nx, ny, 20, checkpoint_every=6)
    v = ri.direction(len(z0), nx, ny, 1)
    lam = ri.direction(len(z0), nx, ny, 2)
    _, jv = gpu_jvp(pr, z0, v)
    jtl = gpu_vjp(pr, z0, lam)
    lhs = sum(float(np.sum(a * b)) for a, b in zip(lam, jv))
    rhs = sum(float(np.sum(a * b)) for a, b in zip(jtl, v))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


@pytest.mark.parametrize("model,stencil,scheme", [("fk", "lap9", "rk4"), ("bocf", "lap9_aniso", "rush_larsen"),
                                                  ("fhn", "lap9_aniso", "heun")])
@pytest.mark.parametrize("tangent", [False, True])
def test_periodic_batched_equals_single_bitwise(model, stencil, scheme, tangent):
    sizes = [(40, 40), (97, 61), (1, 5), (57, 1), (200, 33)]
    cases = []
    for k, (nx, ny) in enumerate(sizes):
        _, pr, z0 = setup(model, stencil, scheme, nx, ny, 5, seed=k)
        cases.append((pr, z0, ri.direction(len(z0), nx, ny, 50 + k)))
    fields = [dev(z0) for _, z0, _ in cases]
    tans = [dev(v) for _, _, v in cases] if tangent else None
    rd.step_batched([pr for pr, _, _ in cases], fields, tans)
    for k, (pr, z0, v) in enumerate(cases):
        zs, vs = dev(z0), dev(v)
        if tangent:
            rd.jvp(pr, zs, vs)
        else:
            rd.step(pr, zs)
        assert all(np.array_equal(a, b) for a, b in zip(host(fields[k]), host(zs))), k
        if tangent:
            assert all(np.array_equal(a, b) for a, b in zip(host(tans[k]), host(vs))), k
