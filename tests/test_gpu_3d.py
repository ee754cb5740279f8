"""GPU parity of the 3-D stencils (rd_step, rd_jvp, rd_vjp with RD_LAP7/19/27)
against the oracle, through the C ABI, plus properties that hold at any
size: the reduction of a single plane to the 2-D operators, z-invariance,
translation equivariance, a Fourier eigenmode at 256^3, checkpoints and HIP
graph replays."""
import itertools
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1309_1720_amd as rd
import rd_inputs as ri
from rdtest import dev, host, problems, rel_linf

pytestmark = pytest.mark.gpu

TOL = 1e-11
BASE = {"diffusion": "fk_1024_rk4", "barkley": "barkley_1024_rk4_adjoint",
        "fk": "fk_1024_rk4", "bocf": "bocf_2048_aniso_rk4", "fhn": "fhn_256_rk4"}
MODELS = ["diffusion", "barkley", "fk", "bocf", "fhn"]
ST3 = ["lap7", "lap19", "lap27"]


def setup(model, stencil, scheme, nx, ny, nz, steps, bc="noflux", seed=3, **kw):
    w = ri.workload(BASE[model], model=model, stencil=stencil, scheme=scheme, nx=nx, ny=ny, nz=nz, bc=bc,
                    D_perp=None, theta0=0.0, theta1=0.0, **kw)
    po, pr = problems(w, nsteps=steps)
    z0 = ri.random_fields(model, nx, ny, seed, nz=nz)
    return po, pr, z0


def gpu_step(pr, z, checkpoints=None):
    zt = dev(z)
    rd.step(pr, zt, checkpoints)
    return host(zt)


def gpu_jvp(pr, z0, v):
    zt, vt = dev(z0), dev(v)
    rd.jvp(pr, zt, vt)
    return host(zt), host(vt)


@pytest.mark.parametrize("model,stencil,scheme", list(itertools.product(MODELS, ST3, ["euler", "heun", "rk4"])))
def test_3d_step_matches_oracle(model, stencil, scheme):
    """70 x 21 x 13: two strips (one ragged), ragged row groups, several z chunks."""
    po, pr, z0 = setup(model, stencil, scheme, 70, 21, 13, 6)
    ref = oracle.step(po, z0, 6)
    got = gpu_step(pr, z0)
    err = rel_linf(got, ref)
    print(f"3-D {model} {stencil} {scheme}: rel-Linf {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("model,stencil,scheme", [("fk", "lap27", "rk4"), ("bocf", "lap19", "heun"),
                                                  ("fhn", "lap7", "rk4"), ("barkley", "lap19", "euler"),
                                                  ("diffusion", "lap27", "heun")])
def test_3d_periodic_step_matches_oracle(model, stencil, scheme):
    po, pr, z0 = setup(model, stencil, scheme, 70, 21, 13, 6, bc="periodic")
    assert rel_linf(gpu_step(pr, z0), oracle.step(po, z0, 6)) <= TOL


@pytest.mark.parametrize("model,stencil,scheme", list(itertools.product(["fk", "bocf"], ST3,
                                                                         ["rush_larsen", "implicit_euler"])))
def test_3d_gate_schemes_match_oracle(model, stencil, scheme):
    po, pr, z0 = setup(model, stencil, scheme, 70, 21, 13, 6)
    assert rel_linf(gpu_step(pr, z0), oracle.step(po, z0, 6)) <= TOL


@pytest.mark.parametrize("model,stencil,scheme,bc", [
    ("fk", "lap27", "rk4", "noflux"), ("bocf", "lap19", "rk4", "periodic"), ("fhn", "lap7", "heun", "noflux"),
    ("barkley", "lap27", "euler", "periodic"), ("diffusion", "lap19", "rk4", "noflux"),
    ("fk", "lap7", "rush_larsen", "noflux"), ("bocf", "lap27", "implicit_euler", "periodic")])
def test_3d_jvp_matches_oracle(model, stencil, scheme, bc):
    po, pr, z0 = setup(model, stencil, scheme, 66, 9, 7, 5, bc=bc)
    v = ri.direction(len(z0), 66, 9, 11, nz=7)
    _, jv_ref = oracle.jvp(po, z0, v, 5)
    z_gpu, jv_gpu = gpu_jvp(pr, z0, v)
    err = rel_linf(jv_gpu, jv_ref)
    print(f"3-D {model} {stencil} {scheme} {bc}: tangent rel-Linf {err:.3e}")
    assert err <= TOL
    # the state half is the plain step, bit for bit
    assert all(np.array_equal(a, b) for a, b in zip(z_gpu, gpu_step(pr, z0)))


@pytest.mark.parametrize("nx,ny,nz", [(1, 1, 1), (1, 1, 9), (9, 1, 1), (1, 9, 1), (2, 2, 2), (63, 5, 2),
                                      (62, 4, 4), (5, 3, 40)])
@pytest.mark.parametrize("bc", ["noflux", "periodic"])
@pytest.mark.parametrize("model,stencil,scheme", [("fk", "lap27", "rk4"), ("fhn", "lap19", "heun")])
def test_3d_degenerate_and_ragged_grids(nx, ny, nz, bc, model, stencil, scheme):
    po, pr, z0 = setup(model, stencil, scheme, nx, ny, nz, 4, bc=bc)
    assert rel_linf(gpu_step(pr, z0), oracle.step(po, z0, 4)) <= TOL


@pytest.mark.parametrize("st3,st2", [("lap7", "lap5"), ("lap19", "lap9"), ("lap27", "lap9")])
@pytest.mark.parametrize("bc", ["noflux", "periodic"])
def test_single_plane_matches_the_2d_kernel(st3, st2, bc):
    """nz = 1: the 3-D operators reduce to the 5-point and Eq. (6) stencils,
    so the 3-D stage kernels must follow the fused 2-D sweep to rounding."""
    nx, ny = 131, 77
    _, p2 = problems(ri.workload("fk_1024_rk4", stencil=st2, nx=nx, ny=ny, bc=bc), nsteps=20)
    _, p3 = problems(ri.workload("fk_1024_rk4", stencil=st3, nx=nx, ny=ny, nz=1, bc=bc), nsteps=20)
    z2 = ri.random_fields("fk", nx, ny, 4)
    a = gpu_step(p2, z2)
    b = gpu_step(p3, [x[None] for x in z2])
    assert rel_linf([x[0] for x in b], a) <= 1e-13


@pytest.mark.parametrize("bc", ["noflux", "periodic"])
def test_z_invariant_state_stays_z_invariant_bitwise(bc):
    nx, ny, nz = 90, 30, 11
    _, pr, _ = setup("bocf", "lap27", "rk4", nx, ny, nz, 7, bc=bc)
    z2 = ri.random_fields("bocf", nx, ny, 8)
    got = gpu_step(pr, [np.repeat(x[None], nz, axis=0) for x in z2])
    for a in got:
        for k in range(1, nz):
            assert np.array_equal(a[k], a[0])


@pytest.mark.parametrize("model,stencil", [("fk", "lap27"), ("fhn", "lap19"), ("barkley", "lap7")])
def test_3d_periodic_translation_equivariance_bitwise(model, stencil):
    nx, ny, nz = 100, 23, 17
    _, pr, z0 = setup(model, stencil, "rk4", nx, ny, nz, 5, bc="periodic")
    a = gpu_step(pr, z0)
    for sh in ((5, 0, 0), (0, 7, 0), (0, 0, 61), (-3, 11, -40)):
        b = gpu_step(pr, [np.roll(x, sh, axis=(0, 1, 2)) for x in z0])
        for x, y in zip(a, b):
            assert np.array_equal(np.roll(x, sh, axis=(0, 1, 2)), y), sh


def test_3d_reflections_bitwise():
    _, pr, z0 = setup("fk", "lap27", "rk4", 70, 21, 13, 5)
    a = gpu_step(pr, z0)
    for axis in range(3):
        flip = [np.ascontiguousarray(np.flip(x, axis)) for x in z0]
        b = gpu_step(pr, flip)
        for x, y in zip(a, b):
            assert np.array_equal(np.flip(x, axis), y), axis


@pytest.mark.parametrize("stencil", ST3)
def test_fourier_mode_at_256_cubed(stencil):
    """A periodic Fourier mode is an eigenvector of each 3-D operator with
    the eigenvalue D/h^2 (w_f faces + w_e edges + w_c corners) of its symbol
    (faces 2 sum cos - 6, edges 4 sum cos cos - 12, corners 8 prod cos - 8);
    explicit Euler multiplies it by (1 + dt lambda) per step.  Independent of
    the oracle, at a full-size 3-D grid."""
    n, steps = 256, 20
    w = ri.workload("fk_1024_rk4", model="diffusion", stencil=stencil, scheme="euler", nx=n, ny=n, nz=n,
                    bc="periodic")
    _, pr = problems(w, nsteps=steps)
    m = (3, 5, 2)
    ph = [2 * math.pi * k / n for k in m]
    x = np.arange(n)
    mode = (np.cos(ph[2] * x + 0.2)[:, None, None] * np.cos(ph[1] * x + 0.7)[None, :, None]
            * np.cos(ph[0] * x + 0.3)[None, None, :])
    ca, cb, cc = (math.cos(p) for p in ph)
    wf, we, wc = {"lap7": (1.0, 0.0, 0.0), "lap19": (1 / 3, 1 / 6, 0.0), "lap27": (7 / 15, 1 / 10, 1 / 30)}[stencil]
    sym = (wf * (2 * (ca + cb + cc) - 6) + we * (4 * (ca * cb + cb * cc + ca * cc) - 12)
           + wc * (8 * ca * cb * cc - 8))
    lam = pr.D_par / pr.dx ** 2 * sym
    got = gpu_step(pr, [mode])[0]
    assert np.max(np.abs(got - (1.0 + pr.dt * lam) ** steps * mode)) <= 1e-12


def test_3d_checkpoints():
    po, pr, z0 = setup("fk", "lap19", "rk4", 40, 12, 9, 7, checkpoint_every=3)
    nck = rd.checkpoint_count(pr)
    ck = torch.zeros(nck * 3 * pr.cells, dtype=torch.float64, device="cuda")
    final = gpu_step(pr, z0, ck)
    cks = ck.cpu().numpy().reshape(nck, 3, 9, 12, 40)
    for m in range(nck):
        ref = oracle.step(po, z0, 3 * m)
        assert rel_linf(list(cks[m]), ref) <= TOL, m
    assert rel_linf(final, oracle.step(po, z0, 7)) <= TOL


def test_3d_step_graph_replays():
    _, pr, z0 = setup("bocf", "lap27", "rk4", 70, 21, 13, 3)
    z, zr = dev(z0), dev(z0)
    rd.step(pr, dev(z0))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            rd.step(pr, z)
    torch.cuda.current_stream().wait_stream(stream)
    for rep in range(4):
        g.replay()
        torch.rand(1 << 16, dtype=torch.float64, device="cuda").sum()
        rd.step(pr, zr)
        torch.cuda.synchronize()
        assert all(np.array_equal(a, b) for a, b in zip(host(z), host(zr))), rep


@pytest.mark.parametrize("model,stencil,scheme", [("fk", "lap27", "rk4"), ("bocf", "lap19", "rush_larsen"),
                                                  ("fhn", "lap7", "heun")])
@pytest.mark.parametrize("tangent", [False, True])
def test_3d_batched_equals_single_bitwise(model, stencil, scheme, tangent):
    sizes = [(20, 8, 5), (70, 21, 13), (1, 3, 9), (64, 4, 2)]
    cases = []
    for k, (nx, ny, nz) in enumerate(sizes):
        _, pr, z0 = setup(model, stencil, scheme, nx, ny, nz, 4, seed=k)
        cases.append((pr, z0, ri.direction(len(z0), nx, ny, 60 + k, nz=nz)))
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


def gpu_vjp(pr, z0, lam):
    zt = dev(z0)
    ck = torch.zeros(max(rd.checkpoint_count(pr), 1) * pr.nfields * pr.cells, dtype=torch.float64, device="cuda")
    rd.step(pr, zt, ck)
    lt = dev(lam)
    rd.vjp(pr, ck, lt)
    return host(lt)


@pytest.mark.parametrize("model,stencil,scheme", list(itertools.product(MODELS, ST3, ["euler", "heun", "rk4"])))
def test_3d_vjp_matches_oracle(model, stencil, scheme):
    """20 x 9 x 6 (a ragged strip, row groups and z chunks), 5 steps,
    checkpoints every 2 (a ragged last segment)."""
    po, pr, z0 = setup(model, stencil, scheme, 20, 9, 6, 5, checkpoint_every=2)
    lam = ri.direction(len(z0), 20, 9, 21, nz=6)
    ref = oracle.vjp(po, z0, lam, 5, checkpoint_every=2)
    got = gpu_vjp(pr, z0, lam)
    err = rel_linf(got, ref)
    print(f"3-D {model} {stencil} {scheme}: adjoint rel-Linf {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("model,stencil,scheme,bc", [("fk", "lap27", "rush_larsen", "noflux"),
                                                     ("bocf", "lap19", "implicit_euler", "periodic"),
                                                     ("fk", "lap7", "implicit_euler", "noflux"),
                                                     ("bocf", "lap27", "rush_larsen", "noflux")])
def test_3d_vjp_gate_schemes_match_oracle(model, stencil, scheme, bc):
    po, pr, z0 = setup(model, stencil, scheme, 20, 9, 6, 5, bc=bc, checkpoint_every=2)
    lam = ri.direction(len(z0), 20, 9, 23, nz=6)
    ref = oracle.vjp(po, z0, lam, 5, checkpoint_every=2)
    err = rel_linf(gpu_vjp(pr, z0, lam), ref)
    print(f"3-D {model} {stencil} {scheme} {bc}: adjoint rel-Linf {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("model,stencil,bc", [("fk", "lap27", "periodic"), ("fhn", "lap19", "noflux"),
                                              ("bocf", "lap7", "periodic")])
def test_3d_vjp_periodic_and_degenerate(model, stencil, bc):
    for nx, ny, nz in ((1, 1, 1), (9, 1, 2), (66, 5, 3)):
        po, pr, z0 = setup(model, stencil, "rk4", nx, ny, nz, 3, bc=bc, checkpoint_every=2)
        lam = ri.direction(len(z0), nx, ny, 5, nz=nz)
        ref = oracle.vjp(po, z0, lam, 3, checkpoint_every=2)
        assert rel_linf(gpu_vjp(pr, z0, lam), ref) <= TOL, (nx, ny, nz)


@pytest.mark.parametrize("model,stencil,bc", [("fk", "lap27", "noflux"), ("bocf", "lap19", "periodic"),
                                              ("fhn", "lap7", "noflux"), ("barkley", "lap27", "periodic")])
def test_3d_dot_product(model, stencil, bc):
    """<lambda, J v> = <J^T lambda, v> for the GPU tangent and adjoint on 70 x 21 x 13, 12 RK4 steps."""
    nx, ny, nz = 70, 21, 13
    _, pr, z0 = setup(model, stencil, "rk4", nx, ny, nz, 12, bc=bc, checkpoint_every=5)
    v = ri.direction(len(z0), nx, ny, 1, nz=nz)
    lam = ri.direction(len(z0), nx, ny, 2, nz=nz)
    _, jv = gpu_jvp(pr, z0, v)
    jtl = gpu_vjp(pr, z0, lam)
    lhs = sum(float(np.sum(a * b)) for a, b in zip(lam, jv))
    rhs = sum(float(np.sum(a * b)) for a, b in zip(jtl, v))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


def test_3d_autograd_flow_gradient():
    """torch.autograd through rd.flow on a 3-D problem: the gradient of
    L = sum(u(T)^2) equals the oracle's adjoint of 2 u(T)."""
    po, pr, z0 = setup("fhn", "lap19", "rk4", 30, 10, 6, 7, checkpoint_every=3)
    zs = [t.requires_grad_(True) for t in dev(z0)]
    out = rd.flow(pr, *zs)
    loss = (out[0] * out[0]).sum()
    loss.backward()
    zT = oracle.step(po, z0, 7)
    ref = oracle.vjp(po, z0, [2.0 * zT[0], np.zeros_like(zT[1])], 7, checkpoint_every=3)
    assert rel_linf([t.grad.cpu().numpy() for t in zs], ref) <= TOL
