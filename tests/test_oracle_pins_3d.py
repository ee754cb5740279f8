"""Pins of the oracle's 3-D operators (lap7, lap19, lap27) and of the
integrator on 3-D states, against facts fixed by the mathematics: Fourier
and cosine modes as exact eigenvectors with the stencil's symbol, exactness
on quadratics, conservation, symmetry, the isotropy of the leading error,
and the reduction of z-invariant problems to the 2-D operators of Eq. 6 and
the 2-D oracle."""
import math

import numpy as np
import pytest

import oracle
import rd_inputs as ri

ST3 = ("lap7", "lap19", "lap27")
BCS = ("noflux", "periodic")


def symbol(st, a, b, c):
    """(h^2 / D) times the eigenvalue of the stencil for a separable mode with
    per-axis phase steps a, b, c: a shift-pair sum of such a mode is 2 cos(phase)
    times the mode, so faces, edges and corners contribute products of cosines."""
    wf, we, wc = oracle.WEIGHTS_3D[st]
    ca, cb, cc = math.cos(a), math.cos(b), math.cos(c)
    faces = 2.0 * (ca + cb + cc) - 6.0
    edges = 4.0 * (ca * cb + cb * cc + ca * cc) - 12.0
    corners = 8.0 * ca * cb * cc - 8.0
    return wf * faces + we * edges + wc * corners


def prob3(st, bc, nx, ny, nz, model="diffusion", scheme="euler", dx=0.5, dt=0.01, D=1.0):
    return oracle.Problem(model=model, scheme=scheme, stencil=st, nx=nx, ny=ny, nz=nz, dx=dx, dt=dt,
                          D_par=D, bc=bc, params=ri.params_array(model))


def test_weights_are_consistent_and_isotropic():
    for st in ST3:
        wf, we, wc = oracle.WEIGHTS_3D[st]
        assert wf + 4 * we + 4 * wc == pytest.approx(1.0, abs=1e-15)          # second moment = 2
        if st != "lap7":
            assert wf == pytest.approx(2 * we + 8 * wc, abs=1e-15)           # fourth moments isotropic


@pytest.mark.parametrize("st", ST3)
def test_periodic_fourier_modes_are_eigenvectors(st):
    nx, ny, nz = 10, 7, 6
    p = prob3(st, "periodic", nx, ny, nz, dx=0.3, D=1.7)
    for mx, my, mz in ((1, 0, 0), (2, 3, 1), (4, 1, 5), (5, 3, 3)):
        a, b, c = 2 * np.pi * mx / nx, 2 * np.pi * my / ny, 2 * np.pi * mz / nz
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        u = np.cos(a * i + 0.3) * np.cos(b * j + 1.1) * np.cos(c * k - 0.4)
        lam = p.D_par / p.dx ** 2 * symbol(st, a, b, c)
        assert np.max(np.abs(oracle.laplacian(p, u) - lam * u)) <= 1e-12 * max(1.0, abs(lam))


@pytest.mark.parametrize("st", ST3)
def test_noflux_cosine_modes_are_eigenvectors(st):
    """DCT-II modes satisfy the mirror ghost rule u(-1) = u(0), u(n) = u(n-1)
    on every face, edge and corner."""
    nx, ny, nz = 9, 6, 5
    p = prob3(st, "noflux", nx, ny, nz, dx=0.4, D=0.8)
    for mx, my, mz in ((0, 0, 1), (1, 2, 3), (8, 5, 4), (3, 0, 2)):
        a, b, c = np.pi * mx / nx, np.pi * my / ny, np.pi * mz / nz
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        u = np.cos(a * (i + 0.5)) * np.cos(b * (j + 0.5)) * np.cos(c * (k + 0.5))
        lam = p.D_par / p.dx ** 2 * symbol(st, a, b, c)
        assert np.max(np.abs(oracle.laplacian(p, u) - lam * u)) <= 1e-12 * max(1.0, abs(lam))


@pytest.mark.parametrize("st", ST3)
def test_exact_on_quadratics_in_the_interior(st):
    nx, ny, nz = 8, 7, 6
    p = prob3(st, "noflux", nx, ny, nz, dx=0.25, D=1.3)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x, y, z = (i + 0.5) * p.dx, (j + 0.5) * p.dx, (k + 0.5) * p.dx
    u = 1.5 * x * x - 0.7 * y * y + 2.0 * z * z + 0.3 * x * y - 1.1 * y * z + 0.9 * x * z + x - 2 * z
    lap = oracle.laplacian(p, u)[1:-1, 1:-1, 1:-1]
    assert np.max(np.abs(lap - p.D_par * 2.0 * (1.5 - 0.7 + 2.0))) <= 1e-10


@pytest.mark.parametrize("st", ST3)
@pytest.mark.parametrize("bc", BCS)
def test_conservation_and_symmetry(st, bc):
    p = prob3(st, bc, 5, 4, 3, dx=0.5, D=1.0)
    u = np.random.default_rng(3).random(p.shape)
    assert abs(oracle.laplacian(p, u).sum()) <= 1e-12 * np.abs(u).sum() / p.dx ** 2
    L = oracle.laplacian_matrix(p).toarray()
    assert np.allclose(L, L.T, atol=1e-13, rtol=0)
    assert np.allclose(L.sum(axis=0), 0.0, atol=1e-12)


def test_leading_error_is_isotropic_except_for_lap7():
    """Apply the operators to periodic plane waves with the same |k| along
    different lattice directions: (6,0,0), (4,4,2) and (2,4,4) cycles on a
    48^3 grid.  The isotropic stencils agree across directions to O((kh)^6);
    the 7-point operator differs already at O((kh)^4)."""
    n = 48
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    for st in ST3:
        p = prob3(st, "periodic", n, n, n, dx=1.0, D=1.0)
        lams = []
        for m in ((6, 0, 0), (4, 4, 2), (2, 4, 4)):
            ph = 2 * np.pi * (m[0] * i + m[1] * j + m[2] * k) / n
            u = np.exp(1j * ph)
            lu = oracle.laplacian(p, u)
            lams.append(complex(lu[3, 5, 7] / u[3, 5, 7]).real)
        kh2 = (2 * np.pi * 6 / n) ** 2
        spread = (max(lams) - min(lams)) / kh2
        # exact continuous value -kh2; leading correction +kh2^2/12 for every isotropic member
        if st == "lap7":
            assert spread > 2e-2
        else:
            assert spread < 1e-3
            for lam in lams:
                assert abs((lam + kh2) - kh2 * kh2 / 12.0) < 0.05 * kh2 * kh2 / 12.0


@pytest.mark.parametrize("bc", BCS)
def test_single_plane_reduces_to_2d(bc):
    """With nz = 1 and mirrored z-neighbours, lap7 is the 5-point operator and
    lap19, lap27 are the 9-point operator of Eq. 6 (for either x-y boundary)."""
    u = np.random.default_rng(7).random((6, 9))
    p2_5 = oracle.Problem(model="diffusion", scheme="euler", stencil="lap5", nx=9, ny=6, dx=0.3, dt=0.01,
                          D_par=1.1, bc=bc, params=ri.params_array("diffusion"))
    p2_9 = oracle.Problem(model="diffusion", scheme="euler", stencil="lap9", nx=9, ny=6, dx=0.3, dt=0.01,
                          D_par=1.1, bc=bc, params=ri.params_array("diffusion"))
    for st, ref in (("lap7", p2_5), ("lap19", p2_9), ("lap27", p2_9)):
        p3 = oracle.Problem(model="diffusion", scheme="euler", stencil=st, nx=9, ny=6, nz=1, dx=0.3, dt=0.01,
                            D_par=1.1, bc=bc, params=ri.params_array("diffusion"))
        got = oracle.laplacian(p3, u[None])[0]
        assert np.max(np.abs(got - oracle.laplacian(ref, u))) <= 1e-13 * np.abs(u).max() / 0.09


@pytest.mark.parametrize("model,st2,st3", [("fk", "lap9", "lap19"), ("bocf", "lap9", "lap27"),
                                           ("fhn", "lap5", "lap7"), ("barkley", "lap9", "lap27")])
@pytest.mark.parametrize("scheme", ["euler", "heun", "rk4"])
def test_z_invariant_state_evolves_as_the_2d_problem(model, st2, st3, scheme):
    """A state constant along z stays so, and each plane follows the 2-D
    oracle with the corresponding stencil of Eq. 6 (or the 5-point one)."""
    base = {"fk": "fk_1024_rk4", "bocf": "bocf_2048_aniso_rk4", "fhn": "fhn_256_rk4",
            "barkley": "barkley_1024_rk4_adjoint"}[model]
    w = ri.workload(base, model=model, stencil=st2, scheme=scheme, nx=11, ny=8)
    params = ri.params_array(model)
    p2 = oracle.Problem.from_workload(w, params=params)
    p3 = oracle.Problem.from_workload(dict(w, stencil=st3, nz=4), params=params)
    z2 = ri.random_fields(model, 11, 8, 5)
    z3 = [np.repeat(a[None], 4, axis=0) for a in z2]
    r2 = oracle.step(p2, z2, 5)
    r3 = oracle.step(p3, z3, 5)
    for a2, a3 in zip(r2, r3):
        for kz in range(4):
            assert np.max(np.abs(a3[kz] - a2)) <= 1e-13 * max(1.0, np.abs(a2).max())


@pytest.mark.parametrize("st", ST3)
@pytest.mark.parametrize("scheme,R", [("euler", lambda z: 1 + z), ("heun", lambda z: 1 + z + z * z / 2),
                                      ("rk4", lambda z: 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24)])
def test_diffusion_mode_decays_by_the_stability_polynomial(st, scheme, R):
    nx, ny, nz = 8, 6, 5
    p = prob3(st, "noflux", nx, ny, nz, scheme=scheme, dx=0.5, dt=0.02, D=1.0)
    a, b, c = np.pi * 3 / nx, np.pi * 1 / ny, np.pi * 2 / nz
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.cos(a * (i + 0.5)) * np.cos(b * (j + 0.5)) * np.cos(c * (k + 0.5))
    lam = p.D_par / p.dx ** 2 * symbol(st, a, b, c)
    out = oracle.step(p, [u], 7)[0]
    assert np.max(np.abs(out - R(lam * p.dt) ** 7 * u)) <= 1e-13


def test_3d_tangent_and_adjoint_small():
    """JVP against central differences and the dot-product test of JVP and
    VJP on a small 3-D Fenton-Karma problem."""
    w = ri.workload("fk_1024_rk4", stencil="lap27", nx=4, ny=3, nz=3, bc="noflux")
    p = oracle.Problem.from_workload(w, params=ri.params_array("fk"))
    z = ri.random_fields("fk", 4, 3, 1, nz=3)
    v = ri.direction(3, 4, 3, 2, nz=3)
    lam = ri.direction(3, 4, 3, 3, nz=3)
    _, jv = oracle.jvp(p, z, v, 3)
    e = 1e-6
    zp = oracle.step(p, [a + e * b for a, b in zip(z, v)], 3)
    zm = oracle.step(p, [a - e * b for a, b in zip(z, v)], 3)
    fd = [(a - b) / (2 * e) for a, b in zip(zp, zm)]
    assert max(float(np.max(np.abs(a - b))) for a, b in zip(jv, fd)) <= 1e-7
    jtl = oracle.vjp(p, z, lam, 3, checkpoint_every=2)
    lhs = sum(float(np.sum(a * b)) for a, b in zip(lam, jv))
    rhs = sum(float(np.sum(a * b)) for a, b in zip(jtl, v))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_problem_rejects_nz_for_2d_stencils():
    with pytest.raises(ValueError):
        oracle.Problem(model="diffusion", scheme="euler", stencil="lap9", nx=4, ny=4, nz=2, dx=1.0, dt=0.1)
