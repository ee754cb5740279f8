"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms (quadratics, DCT eigenpairs, stability polynomials), invariants
(conservation, symmetry, uniform states), the paper's printed convergence
orders (Table 1), independent formulations (textbook piecewise models,
central finite differences, dense Jacobians) and the smoothed step's facts.
"""
import dataclasses
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import rd_inputs as ri

import conditioning

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def prob(model="diffusion", stencil="lap5", scheme="euler", nx=12, ny=10, dx=0.5, dt=0.01,
         **kw):
    params = kw.pop("params", tuple(ri.params_array(model)))
    return oracle.Problem(model=model, stencil=stencil, scheme=scheme, nx=nx, ny=ny, dx=dx,
                          dt=dt, params=params, **kw)


def grid(nx, ny, dx):
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    return np.meshgrid(x, y)  # X[j, i] = x_i


def flat(z):
    return np.concatenate([np.ravel(a) for a in z])


# ---------------------------------------------------------------------------
# Stencils (Sect. 3, Eq. 6; Fig. 1)
# ---------------------------------------------------------------------------

QUAD = (3.0, -2.0, 5.0, 1.0, -4.0, 7.0)


def quadratic(X, Y, a, b, c, d, e, f):
    return a * X * X + b * X * Y + c * Y * Y + d * X + e * Y + f


def test_quadratic_exact_lap5():
    nx, ny, dx, D = 11, 9, 0.5, 1.5
    X, Y = grid(nx, ny, dx)
    u = quadratic(X, Y, *QUAD)
    lap = oracle.laplacian(prob(stencil="lap5", nx=nx, ny=ny, dx=dx, D_par=D), u)
    a, _, c = QUAD[:3]
    # dyadic inputs: exact arithmetic, bitwise equality at interior cells
    assert np.all(lap[1:-1, 1:-1] == D * (2 * a + 2 * c))


def test_quadratic_lap9():
    nx, ny, dx, D = 11, 9, 0.5, 1.5
    X, Y = grid(nx, ny, dx)
    u = quadratic(X, Y, *QUAD)
    lap = oracle.laplacian(prob(stencil="lap9", nx=nx, ny=ny, dx=dx, D_par=D), u)
    a, _, c = QUAD[:3]
    exact = D * (2 * a + 2 * c)
    assert np.max(np.abs(lap[1:-1, 1:-1] - exact)) <= 4e-16 * abs(exact) * 8


@pytest.mark.parametrize("theta", [0.0, 0.4, -1.0, math.pi / 2])
def test_quadratic_aniso_constant_angle(theta):
    nx, ny, dx = 11, 9, 0.5
    Dp, Dq = 1.25, 0.375
    X, Y = grid(nx, ny, dx)
    u = quadratic(X, Y, *QUAD)
    p = prob(stencil="lap9_aniso", nx=nx, ny=ny, dx=dx, D_par=Dp, D_perp=Dq,
             theta0=theta, theta1=theta)
    lap = oracle.laplacian(p, u)
    c_, s_ = math.cos(theta), math.sin(theta)
    dxx = Dq + (Dp - Dq) * c_ * c_
    dxy = (Dp - Dq) * c_ * s_
    dyy = Dq + (Dp - Dq) * s_ * s_
    a, b, c = QUAD[:3]
    exact = 2 * a * dxx + 2 * b * dxy + 2 * c * dyy
    assert np.max(np.abs(lap[1:-1, 1:-1] - exact)) <= 1e-13 * abs(exact)


def dct_mode(nx, ny, m, n):
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    return np.cos(math.pi * m * (i + 0.5) / nx) * np.cos(math.pi * n * (j + 0.5) / ny)


def dct_eigenvalue(stencil, c, nx, ny, m, n):
    mu_m = -4.0 * math.sin(math.pi * m / (2 * nx)) ** 2
    mu_n = -4.0 * math.sin(math.pi * n / (2 * ny)) ** 2
    if stencil == "lap5":
        return c * (mu_m + mu_n)
    return c * ((mu_m + mu_n) + mu_m * mu_n / 6.0)


@pytest.mark.parametrize("stencil", ["lap5", "lap9"])
@pytest.mark.parametrize("mn", [(0, 1), (1, 0), (3, 2), (12, 9), (5, 7), (0, 0)])
def test_dct_modes_are_eigenvectors(stencil, mn):
    """Half-sample-mirrored ghosts make cos modes exact eigenvectors,
    edges and corners included (pins the ghost rule of Fig. 1 and Eq. 6)."""
    nx, ny, dx, D = 13, 10, 0.4, 0.7
    m, n = mn
    phi = dct_mode(nx, ny, m, n)
    c = D / (dx * dx)
    lam = dct_eigenvalue(stencil, c, nx, ny, m, n)
    lap = oracle.laplacian(prob(stencil=stencil, nx=nx, ny=ny, dx=dx, D_par=D), phi)
    assert np.max(np.abs(lap - lam * phi)) <= 1e-13 * max(abs(lam), c)


@pytest.mark.parametrize("stencil", ["lap5", "lap9"])
@pytest.mark.parametrize("scheme,R", [
    ("euler", lambda x: 1 + x),
    ("heun", lambda x: 1 + x + x * x / 2),
    ("rk4", lambda x: 1 + x + x * x / 2 + x ** 3 / 6 + x ** 4 / 24),
])
def test_pure_diffusion_mode_decay(stencil, scheme, R):
    """z_n = R(lambda dt)^n phi: pins each scheme's stability polynomial."""
    nx, ny, dx, D, dt, steps = 12, 9, 0.5, 1.0, 0.02, 50
    phi = dct_mode(nx, ny, 3, 2)
    p = prob(stencil=stencil, scheme=scheme, nx=nx, ny=ny, dx=dx, D_par=D, dt=dt)
    lam = dct_eigenvalue(stencil, D / dx ** 2, nx, ny, 3, 2)
    out = oracle.step(p, [phi], steps)[0]
    expect = R(lam * dt) ** steps * phi
    assert np.max(np.abs(out - expect)) <= 1e-13 * np.max(np.abs(expect))


@pytest.mark.parametrize("stencil", ["lap5", "lap9"])
@pytest.mark.parametrize("scheme,R", [
    ("euler", lambda x: 1 + x),
    ("heun", lambda x: 1 + x + x * x / 2),
    ("rk4", lambda x: 1 + x + x * x / 2 + x ** 3 / 6 + x ** 4 / 24),
])
def test_fhn_second_field_diffuses_with_delta(stencil, scheme, R):
    """Eq. (3) with eps = 0 leaves v alone with delta lap v: a DCT mode of v
    decays as R(delta lambda dt)^n, whatever u does (pins v's diffusivity)."""
    nx, ny, dx, dt, steps, delta = 12, 9, 0.5, 0.01, 40, 1.5
    phi = dct_mode(nx, ny, 2, 3)
    p = prob(model="fhn", stencil=stencil, scheme=scheme, nx=nx, ny=ny, dx=dx, dt=dt,
             params=(delta, 0.0, 1.5, -0.1))
    lam = dct_eigenvalue(stencil, delta / dx ** 2, nx, ny, 2, 3)
    u0 = 0.3 * np.cos(np.arange(nx)[None, :] * 0.7) * np.ones((ny, 1))
    out = oracle.step(p, [u0, phi], steps)[1]
    expect = R(lam * dt) ** steps * phi
    assert np.max(np.abs(out - expect)) <= 1e-13 * np.max(np.abs(expect))


def test_fhn_brute_force_euler_step():
    """Eq. (3), one explicit Euler step with the 5-point stencil and mirrored
    ghosts written as scalar loops on a 5 x 4 grid: the oracle's step agrees
    bit for bit."""
    nx, ny, dx, dt = 5, 4, 0.3, 0.001
    delta, eps, a1, a0 = 1.5, 0.05, 1.5, -0.1
    rng = np.random.default_rng(7)
    u = (rng.random((ny, nx)) - 0.5) * 2.0
    v = (rng.random((ny, nx)) - 0.5)
    c_u, c_v = 1.0 / (dx * dx), (1.0 * delta) / (dx * dx)

    def at(a, j, i):
        return a[min(max(j, 0), ny - 1)][min(max(i, 0), nx - 1)]

    un, vn = np.empty_like(u), np.empty_like(v)
    for j in range(ny):
        for i in range(nx):
            lu = c_u * (((at(u, j, i - 1) + at(u, j, i + 1)) + (at(u, j - 1, i) + at(u, j + 1, i))) - 4.0 * u[j, i])
            lv = c_v * (((at(v, j, i - 1) + at(v, j, i + 1)) + (at(v, j - 1, i) + at(v, j + 1, i))) - 4.0 * v[j, i])
            fu = (u[j, i] - v[j, i]) - (u[j, i] * u[j, i]) * u[j, i]
            fv = eps * ((u[j, i] - a1 * v[j, i]) - a0)
            un[j, i] = u[j, i] + dt * (lu + fu)
            vn[j, i] = v[j, i] + dt * (lv + fv)
    p = prob(model="fhn", stencil="lap5", scheme="euler", nx=nx, ny=ny, dx=dx, dt=dt,
             params=(delta, eps, a1, a0))
    out = oracle.step(p, [u, v], 1)
    assert np.array_equal(out[0], un) and np.array_equal(out[1], vn)


@pytest.mark.parametrize("stencil", ["lap5", "lap9", "lap9_aniso"])
@pytest.mark.parametrize("scheme", ["euler", "rk4"])
def test_pure_diffusion_conserves_sum(stencil, scheme):
    """No-flux boundaries conserve the plain field sum (Eq. 2)."""
    nx, ny = 23, 17
    p = prob(stencil=stencil, scheme=scheme, nx=nx, ny=ny, dx=0.025, dt=0.05,
             D_par=0.001171, D_perp=0.001171 / 4, theta0=-math.pi / 3, theta1=math.pi / 3)
    u0 = ri.diffusion_ic(nx, ny, 7)
    u1 = oracle.step(p, u0, 1000)[0]
    assert abs(u1.sum() - u0[0].sum()) <= 1e-13 * abs(u0[0].sum())
    assert np.max(np.abs(u1 - u0[0])) > 1e-3  # it did diffuse


@pytest.mark.parametrize("stencil", ["lap5", "lap9", "lap9_aniso"])
def test_sparse_operator_matches_stencil(stencil):
    nx, ny = 5, 4
    p = prob(stencil=stencil, nx=nx, ny=ny, dx=0.3, D_par=0.9, D_perp=0.2,
             theta0=-0.8, theta1=1.1)
    L = oracle.laplacian_matrix(p).toarray()
    dense = np.zeros_like(L)
    for k in range(nx * ny):
        e = np.zeros(nx * ny)
        e[k] = 1.0
        dense[:, k] = oracle.laplacian(p, e.reshape(ny, nx)).ravel()
    assert np.max(np.abs(L - dense)) <= 1e-14 * np.max(np.abs(L))
    one = np.ones(nx * ny)
    assert np.max(np.abs(L @ one)) <= 1e-14 * np.max(np.abs(L))   # balanced rows
    assert np.max(np.abs(one @ L)) <= 1e-14 * np.max(np.abs(L))   # conservative columns
    if stencil != "lap9_aniso":
        assert np.array_equal(L, L.T)                              # symmetric operator


def test_aniso_second_order_against_analytic_divergence():
    """Interior cells converge to div(D(x) grad u) at order 2 for smooth u
    and a fibre angle linear in x."""
    Dp, Dq, th0, th1 = 1.0, 0.25, -math.pi / 3, math.pi / 3
    errs = []
    for n in (16, 32, 64):
        Lx = 1.0
        dx = Lx / n
        X, Y = grid(n, n, dx)
        al, be = 2.1, 1.3
        u = np.sin(al * X + 0.3) * np.cos(be * Y - 0.2)
        ux = al * np.cos(al * X + 0.3) * np.cos(be * Y - 0.2)
        uy = -be * np.sin(al * X + 0.3) * np.sin(be * Y - 0.2)
        uxx = -al * al * u
        uyy = -be * be * u
        uxy = -al * be * np.cos(al * X + 0.3) * np.sin(be * Y - 0.2)
        th = th0 + (th1 - th0) * X / Lx
        dth = (th1 - th0) / Lx
        dd = Dp - Dq
        dxx = Dq + dd * np.cos(th) ** 2
        dxy = dd * np.cos(th) * np.sin(th)
        dyy = Dq + dd * np.sin(th) ** 2
        dxx_x = -dd * np.sin(2 * th) * dth
        dxy_x = dd * np.cos(2 * th) * dth
        exact = dxx_x * ux + dxx * uxx + dxy_x * uy + 2 * dxy * uxy + dyy * uyy
        p = prob(stencil="lap9_aniso", nx=n, ny=n, dx=dx, D_par=Dp, D_perp=Dq,
                 theta0=th0, theta1=th1)
        lap = oracle.laplacian(p, u)
        errs.append(np.max(np.abs(lap - exact)[2:-2, 2:-2]))
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(1.8 < o < 2.3 for o in orders), orders


@pytest.mark.parametrize("stencil", ["lap5", "lap9", "lap9_aniso"])
def test_uniform_field_has_zero_diffusion(stencil):
    p = prob(stencil=stencil, nx=9, ny=7, D_par=0.9, D_perp=0.3, theta0=0.2, theta1=1.4)
    u = np.full((7, 9), 0.734512)
    assert np.all(oracle.laplacian(p, u) == 0.0)


# ---------------------------------------------------------------------------
# Smoothed step (Sect. 2)
# ---------------------------------------------------------------------------

def test_smooth_step_facts():
    k = ri.STEP_K
    H = lambda x: oracle.smooth_step(np.asarray(x, dtype=np.float64), k)
    assert H(0.0) == 0.5
    assert H(0.5 / k + 1e-12) == 1.0 and H(-0.5 / k - 1e-12) == 0.0
    assert H(10.0) == 1.0 and H(-10.0) == 0.0
    x = np.linspace(-1.0 / k, 1.0 / k, 2001)
    h = H(x)
    assert np.all(np.diff(h) >= 0)                         # monotone
    assert np.max(np.abs(h + H(-x) - 1.0)) <= 2.3e-16      # odd symmetry about 1/2
    # the paper's printed form, (3 - 2kx - 1)(kx + 0.5)^2 on |kx| <= 1/2
    mid = np.abs(k * x) <= 0.5
    literal = (3.0 - 2.0 * k * x - 1.0) * (k * x + 0.5) ** 2
    assert np.max(np.abs(h[mid] - literal[mid])) <= 4e-16
    # width 1/k ~ 0.035 quoted in the text
    assert abs(1.0 / k - 0.035) < 5e-4
    # C1: derivative vanishes at both ends of the transition (one-sided slopes)
    e = 1e-7
    for x0 in (-0.5 / k, 0.5 / k):
        # slopes over e shrink like 3 k^2 e: no jump in the first derivative
        assert abs(float(H(x0 + e) - H(x0)) / e) < 4 * k * k * e
        assert abs(float(H(x0) - H(x0 - e)) / e) < 4 * k * k * e
    # slope at the centre: dH/dx = 6k t(1-t) = 1.5 k
    assert abs(float(H(e) - H(-e)) / (2 * e) - 1.5 * k) < 1e-5 * k


def test_sharp_step_limit():
    H = lambda x: oracle.smooth_step(np.asarray(x, dtype=np.float64), math.inf)
    assert H(0.0) == 1.0 and H(-1e-300) == 0.0 and H(3.0) == 1.0


# ---------------------------------------------------------------------------
# Reactions: independent textbook forms away from the thresholds
# ---------------------------------------------------------------------------

def react(model, u, *h):
    p = prob(model=model, nx=1, ny=1)
    z = [np.full((1, 1), float(a)) for a in (u,) + h]
    return [float(a[0, 0]) for a in oracle.reaction(p, z)]


def test_barkley_cubic_roots_and_leading_coefficient():
    a, b, eps = (ri.BARKLEY_PARAMS[n] for n in ("a", "b", "eps"))
    rng = np.random.default_rng(0)
    for v in rng.random(5):
        uth = (v + b) / a
        assert react("barkley", 0.0, v)[0] == 0.0
        assert react("barkley", 1.0, v)[0] == 0.0
        assert abs(react("barkley", uth, v)[0]) < 1e-13
        big = 1e4
        assert abs(react("barkley", big, v)[0] / big ** 3 + 1.0 / eps) < 1e-3 / eps
        assert react("barkley", 0.3, v)[1] == 0.3 - v


def fk_textbook(u, v, w, P):
    """Fenton & Karma (1998) with sharp Heaviside gates, written piecewise."""
    jsi = -w * (1.0 + math.tanh(P["k_si"] * (u - P["u_c_si"]))) / (2.0 * P["tau_si"])
    if u >= P["u_c"]:
        jfi = -v * (1.0 - u) * (u - P["u_c"]) / P["tau_d"]
        jso = 1.0 / P["tau_r"]
        dv = -v / P["tau_v_plus"]
        dw = -w / P["tau_w_plus"]
    else:
        jfi = 0.0
        jso = u / P["tau_0"]
        tau_vm = P["tau_v1_minus"] if u >= P["u_v"] else P["tau_v2_minus"]
        dv = (1.0 - v) / tau_vm
        dw = (1.0 - w) / P["tau_w_minus"]
    return [-(jfi + jso + jsi), dv, dw]


@pytest.mark.parametrize("u", [0.0, 0.01, 0.03, 0.08, 0.1, 0.16, 0.4, 0.9, 1.0])
def test_fk_matches_textbook_away_from_thresholds(u):
    P = ri.FK_PARAMS
    rng = np.random.default_rng(int(u * 1000))
    for v, w in rng.random((3, 2)):
        got = react("fk", u, v, w)
        exp = fk_textbook(u, v, w, P)
        for g, e in zip(got, exp):
            assert abs(g - e) <= 1e-14 * max(1.0, abs(e)), (u, v, w, got, exp)


def bocf_textbook(u, v, w, s, P):
    """Bueno-Orovio, Cherry & Fenton (2008) with sharp Heaviside gates."""
    th = lambda x: 1.0 if x >= 0 else 0.0
    t_vm = (1 - th(u - P["theta_v_minus"])) * P["tau_v1_minus"] + th(u - P["theta_v_minus"]) * P["tau_v2_minus"]
    t_wm = P["tau_w1_minus"] + (P["tau_w2_minus"] - P["tau_w1_minus"]) * (1 + math.tanh(P["k_w_minus"] * (u - P["u_w_minus"]))) / 2
    t_so = P["tau_so1"] + (P["tau_so2"] - P["tau_so1"]) * (1 + math.tanh(P["k_so"] * (u - P["u_so"]))) / 2
    t_s = (1 - th(u - P["theta_w"])) * P["tau_s1"] + th(u - P["theta_w"]) * P["tau_s2"]
    t_o = (1 - th(u - P["theta_o"])) * P["tau_o1"] + th(u - P["theta_o"]) * P["tau_o2"]
    v_inf = 1.0 if u < P["theta_v_minus"] else 0.0
    w_inf = (1 - th(u - P["theta_o"])) * (1 - u / P["tau_w_inf"]) + th(u - P["theta_o"]) * P["w_inf_star"]
    jfi = -v * th(u - P["theta_v"]) * (u - P["theta_v"]) * (P["u_u"] - u) / P["tau_fi"]
    jso = (u - P["u_o"]) * (1 - th(u - P["theta_w"])) / t_o + th(u - P["theta_w"]) / t_so
    jsi = -th(u - P["theta_w"]) * w * s / P["tau_si"]
    dv = (1 - th(u - P["theta_v"])) * (v_inf - v) / t_vm - th(u - P["theta_v"]) * v / P["tau_v_plus"]
    dw = (1 - th(u - P["theta_w"])) * (w_inf - w) / t_wm - th(u - P["theta_w"]) * w / P["tau_w_plus"]
    ds = ((1 + math.tanh(P["k_s"] * (u - P["u_s"]))) / 2 - s) / t_s
    return [-(jfi + jso + jsi), dv, dw, ds]


@pytest.mark.parametrize("u", [-0.05, 0.03, 0.05, 0.1, 0.2, 0.25, 0.5, 1.0, 1.5])
def test_bocf_matches_textbook_away_from_thresholds(u):
    P = ri.BOCF_PARAMS
    rng = np.random.default_rng(int((u + 1) * 1000))
    for v, w, s in rng.random((3, 3)):
        got = react("bocf", u, v, w, s)
        exp = bocf_textbook(u, v, w, s, P)
        for g, e in zip(got, exp):
            assert abs(g - e) <= 1e-13 * max(1.0, abs(e)), (u, got, exp)


# ---------------------------------------------------------------------------
# Time stepping: uniform states, convergence orders (Table 1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("model,z0,T,dt", [
    ("barkley", (0.8, 0.1), 1.0, 0.005),
    ("fk", (0.3, 1.0, 1.0), 10.0, 0.01),
    ("bocf", (0.5, 1.0, 1.0, 0.0), 10.0, 0.01),
    ("fhn", (0.7, -0.2), 5.0, 0.005),
])
def test_uniform_state_follows_the_ode(model, z0, T, dt):
    """A spatially uniform state stays exactly uniform and follows the local
    ODE; checked against an independent high-order adaptive integrator."""
    p = prob(model=model, scheme="rk4", stencil="lap9", nx=5, ny=4, dt=dt)
    z = [np.full((4, 5), x) for x in z0]
    out = oracle.step(p, z, int(round(T / dt)))
    for a in out:
        assert np.all(a == a[0, 0])
    p1 = prob(model=model, nx=1, ny=1)

    def f(t, y):
        return [float(r[0, 0]) for r in oracle.reaction(p1, [np.full((1, 1), a) for a in y])]

    ref = solve_ivp(f, (0.0, T), list(z0), method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    got = np.array([a[0, 0] for a in out])
    assert np.max(np.abs(got - ref)) <= 1e-8 * max(1.0, np.max(np.abs(ref)))


def richardson_orders(model, stencil, scheme, n, T, dt0, levels, step_k=ri.STEP_K):
    base = {"barkley": "barkley_128_euler", "fk": "fk_1024_rk4", "bocf": "bocf_2048_aniso_rk4",
            "fhn": "fhn_256_rk4"}[model]
    w = ri.workload(base, nx=n, ny=n, stencil=stencil, scheme=scheme)
    z0 = ri.initial_condition(w)
    sols = []
    for l in range(levels):
        dt = dt0 / 2 ** l
        p = oracle.Problem.from_workload(dict(w, dt=dt), params=ri.params_array(model),
                                         step_k=step_k)
        sols.append(flat(oracle.step(p, z0, int(round(T / dt)))))
    e = [np.linalg.norm(sols[k] - sols[k + 1]) / np.linalg.norm(sols[k + 1])
         for k in range(levels - 1)]
    return [math.log2(e[k] / e[k + 1]) for k in range(len(e) - 1)]


def table1():
    with open(os.path.join(GOLDEN, "table1_orders.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("scheme,key", [("euler", "explicit_euler"), ("heun", "heun"), ("rk4", "rk4")])
def test_fhn_orders_match_table1(scheme, key):
    """FitzHugh-Nagumo (Eq. 3) with the paper's dx = 0.04: Table 1 reports
    the theoretical orders 1, 2 and 4."""
    expected = table1()["observed"][key][0]
    orders = richardson_orders("fhn", "lap9", scheme, 32, 0.06, 3e-4, 5)
    assert abs(orders[-1] - expected) < 0.15, orders


@pytest.mark.parametrize("scheme,key", [("euler", "explicit_euler"), ("heun", "heun"), ("rk4", "rk4")])
def test_barkley_orders_match_table1_polynomial_column(scheme, key):
    """Polynomial reaction: the theoretical order, as for FitzHugh-Nagumo."""
    expected = table1()["observed"][key][0]
    orders = richardson_orders("barkley", "lap5", scheme, 32, 1.0, 0.02, 5)
    assert abs(orders[-1] - expected) < 0.15, orders


@pytest.mark.parametrize("scheme,key", [("euler", "explicit_euler"), ("heun", "heun"), ("rk4", "rk4")])
def test_bocf_orders_match_table1(scheme, key):
    """H_k-gated Bueno-Orovio model: Table 1 reports 1, 2 and 3 (not 4) for RK4."""
    expected = table1()["observed"][key][2]
    orders = richardson_orders("bocf", "lap9_aniso", scheme, 24, 8.0, 0.05, 5)
    assert abs(orders[-1] - expected) < 0.2, orders


@pytest.mark.parametrize("scheme,key", [("rush_larsen", "rush_larsen"), ("implicit_euler", "implicit_euler")])
def test_bocf_gate_schemes_orders_match_table1(scheme, key):
    """Table 1: Rush-Larsen and implicit Euler (gates only) are first order."""
    expected = table1()["observed"][key][2]
    orders = richardson_orders("bocf", "lap9_aniso", scheme, 24, 8.0, 0.05, 5)
    assert abs(orders[-1] - expected) < 0.15, orders


@pytest.mark.parametrize("scheme", ["rush_larsen", "implicit_euler"])
def test_gate_schemes_exact_on_resting_bocf(scheme):
    """At rest (u = u_o = 0) the Bueno-Orovio voltage rate vanishes, so u stays
    0 and each gate obeys dg/dt = alpha g + beta with constant coefficients.
    Rush-Larsen reproduces the exact solution g_inf + (g0 - g_inf) e^{alpha t}
    for any dt; implicit Euler its closed form g_inf + (g0 - g_inf) / (1 -
    alpha dt)^n.  Also pins that each gate's rate is affine in the gate."""
    dt, n = 0.7, 25
    p = prob(model="bocf", scheme=scheme, stencil="lap5", nx=5, ny=4, dt=dt)
    z0 = [np.full((4, 5), x) for x in (0.0, 0.3, 0.6, 0.8)]
    coef = oracle.gate_coefficients(p, z0)
    rates = oracle.reaction(p, z0)
    out = oracle.step(p, z0, n)
    assert np.all(out[0] == 0.0)
    for g in (1, 2, 3):
        a, b = coef[g]
        assert np.max(np.abs(rates[g] - (a * z0[g] + b))) <= 1e-16
        a, b = float(a[0, 0]), float(b[0, 0])
        ginf, g0 = -b / a, float(z0[g][0, 0])
        if scheme == "rush_larsen":
            expect = ginf + (g0 - ginf) * math.exp(a * n * dt)
        else:
            expect = ginf + (g0 - ginf) / (1.0 - a * dt) ** n
        assert np.max(np.abs(out[g] - expect)) <= 1e-14, (scheme, g)


def test_sharp_heaviside_drops_rk4_to_first_order():
    """With the discontinuous step (k = inf) RK4 loses its order: the reason
    the paper smooths the step for derivative-based work."""
    orders = richardson_orders("fk", "lap9", "rk4", 24, 6.0, 0.1, 4, step_k=math.inf)
    assert orders[-1] < 1.5, orders


# ---------------------------------------------------------------------------
# Tangent-linear and adjoint
# ---------------------------------------------------------------------------

CASES = [
    ("barkley", "lap5", "rk4"), ("barkley", "lap5", "euler"), ("fk", "lap9", "rk4"),
    ("fk", "lap9", "heun"), ("bocf", "lap9_aniso", "rk4"), ("bocf", "lap9", "euler"),
    ("diffusion", "lap9_aniso", "rk4"), ("fhn", "lap9", "rk4"), ("fhn", "lap5", "heun"),
]


def case_problem(model, stencil, scheme, nx=14, ny=11):
    base = {"barkley": "barkley_1024_rk4_adjoint", "fk": "fk_1024_rk4",
            "bocf": "bocf_2048_aniso_rk4", "diffusion": "bocf_2048_aniso_rk4", "fhn": "fhn_256_rk4"}[model]
    w = ri.workload(base, nx=nx, ny=ny, model=model, stencil=stencil, scheme=scheme)
    if model == "diffusion":
        w["ic"] = "diffusion"
    p = oracle.Problem.from_workload(w, params=ri.params_array(model))
    z0 = ri.initial_condition(w) if model != "bocf" else ri.random_fields("bocf", nx, ny, 3)
    return p, z0


@pytest.mark.parametrize("model,stencil,scheme", CASES)
def test_jvp_matches_central_differences(model, stencil, scheme):
    p, z0 = case_problem(model, stencil, scheme)
    nv = len(z0)
    v = ri.direction(nv, p.nx, p.ny, 11)
    steps = 10
    _, jv = oracle.jvp(p, z0, v, steps)
    eps = 1e-6
    zp = oracle.step(p, [a + eps * b for a, b in zip(z0, v)], steps)
    zm = oracle.step(p, [a - eps * b for a, b in zip(z0, v)], steps)
    fd = (flat(zp) - flat(zm)) / (2 * eps)
    assert np.linalg.norm(fd - flat(jv)) <= 1e-7 * np.linalg.norm(flat(jv))


@pytest.mark.parametrize("model,stencil,scheme", CASES)
def test_dot_product_jvp_vjp(model, stencil, scheme):
    """<J v, w> = <v, J^T w> over a multi-step flow (adjoint vs tangent)."""
    p, z0 = case_problem(model, stencil, scheme)
    nv = len(z0)
    v = ri.direction(nv, p.nx, p.ny, 21)
    w = ri.direction(nv, p.nx, p.ny, 22)
    steps = 12
    _, jv = oracle.jvp(p, z0, v, steps)
    jtw = oracle.vjp(p, z0, w, steps, checkpoint_every=5)
    a = float(flat(jv) @ flat(w))
    b = float(flat(v) @ flat(jtw))
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


@pytest.mark.parametrize("model,stencil,scheme", [("barkley", "lap9", "rk4"), ("fk", "lap5", "heun"),
                                                  ("bocf", "lap9_aniso", "rk4"), ("fhn", "lap9", "rk4"),
                                                  ("fhn", "lap9_aniso", "euler")])
def test_vjp_equals_transpose_of_dense_jacobian(model, stencil, scheme):
    p, z0 = case_problem(model, stencil, scheme, nx=4, ny=3)
    nv, n = len(z0), 12
    steps = 3
    J = np.zeros((nv * n, nv * n))
    for k in range(nv * n):
        e = np.zeros(nv * n)
        e[k] = 1.0
        _, jv = oracle.jvp(p, z0, [a.reshape(3, 4) for a in np.split(e, nv)], steps)
        J[:, k] = flat(jv)
    lam = ri.direction(nv, 4, 3, 5)
    got = flat(oracle.vjp(p, z0, lam, steps, checkpoint_every=2))
    assert np.max(np.abs(got - J.T @ flat(lam))) <= 1e-13 * np.max(np.abs(J.T @ flat(lam)))


def test_jvp_is_linear():
    p, z0 = case_problem("fk", "lap9", "rk4")
    v = ri.direction(3, p.nx, p.ny, 1)
    w = ri.direction(3, p.nx, p.ny, 2)
    _, a = oracle.jvp(p, z0, v, 5)
    _, b = oracle.jvp(p, z0, w, 5)
    _, c = oracle.jvp(p, z0, [x + 2.0 * y for x, y in zip(v, w)], 5)
    assert np.max(np.abs(flat(c) - (flat(a) + 2.0 * flat(b)))) <= 1e-13 * np.max(np.abs(flat(c)))


def test_fd_error_v_curve():
    """Central-difference JVP error ~ A eps^2 + B/eps: falls with eps at first,
    rises again once rounding dominates; its best is near 1e-9 relative."""
    p, z0 = case_problem("barkley", "lap5", "rk4", nx=16, ny=16)
    v = ri.direction(2, 16, 16, 3)
    steps = 20
    _, jv = oracle.jvp(p, z0, v, steps)
    ref = flat(jv)
    errs = {}
    for eps in (1e-9, 1e-8, 1e-7, 1e-6, 1e-5, 1e-4, 1e-3):
        zp = oracle.step(p, [a + eps * b for a, b in zip(z0, v)], steps)
        zm = oracle.step(p, [a - eps * b for a, b in zip(z0, v)], steps)
        errs[eps] = np.linalg.norm((flat(zp) - flat(zm)) / (2 * eps) - ref) / np.linalg.norm(ref)
    assert errs[1e-3] / errs[1e-4] > 30           # truncation regime, slope ~2
    assert errs[1e-9] > errs[1e-7]                # rounding regime
    assert min(errs.values()) < 1e-8


@pytest.mark.parametrize("horizon", [250, 2000])
def test_fd_gradient_agrees_with_exact_adjoint_over_long_horizons(horizon):
    """The adjoint workload's loss L = dx^2 sum u(T)^2 (Barkley, 5-point,
    RK4, dt = 0.02, the cross-field spiral seed) on a 40^2 grid: the central
    difference (L(z + e v) - L(z - e v)) / 2e, with the loss difference summed
    cell by cell as dx^2 sum (u+ - u-)(u+ + u-), against <g, v> of the
    oracle's exact adjoint gradient g, in four seeded unit directions.  Up to
    2000 steps (40 time units, a dozen spiral turns) the two agree to 1e-7 of
    sigma = ||g|| / sqrt(N) at e = 1e-5: on this grid the loss is smooth on
    that scale, so the exact gradient and the difference quotient check each
    other over long horizons.  (On the workload's 1024^2 grid they do so only
    up to a few hundred steps; beyond, the quotients stray by ~1e-2 sigma at
    every e from 1e-7 to 1e-4 while the exact gradient still matches the
    oracle's to rounding.)"""
    n = 40
    w = ri.workload("barkley_1024_rk4_adjoint", nx=n, ny=n, nsteps=horizon)
    p = oracle.Problem.from_workload(w, params=ri.params_array("barkley"))
    z0 = ri.initial_condition(w)
    zT = oracle.step(p, z0, horizon)
    g = oracle.vjp(p, z0, [2.0 * w["dx"] ** 2 * zT[0], np.zeros_like(zT[1])], horizon,
                   checkpoint_every=64)
    sigma = np.linalg.norm(flat(g)) / math.sqrt(flat(g).size)
    eps = 1e-5
    worst = 0.0
    for seed in range(7000, 7004):
        v = ri.direction(2, n, n, seed)
        exact = float(flat(g) @ flat(v))
        up = oracle.step(p, [a + eps * b for a, b in zip(z0, v)], horizon)[0]
        um = oracle.step(p, [a - eps * b for a, b in zip(z0, v)], horizon)[0]
        fd = w["dx"] ** 2 * float(np.sum((up - um) * (up + um))) / (2 * eps)
        worst = max(worst, abs(fd - exact) / sigma)
    assert worst <= 1e-7, worst


# ---------------------------------------------------------------------------
# Symmetries and inputs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("model,stencil", [("barkley", "lap5"), ("fk", "lap9"), ("bocf", "lap9")])
def test_reflection_symmetry_bitwise(model, stencil):
    p, _ = case_problem(model, stencil, "rk4", nx=13, ny=9)
    z0 = ri.random_fields(model, 13, 9, 4)
    a = oracle.step(p, z0, 6)
    b = oracle.step(p, [x[:, ::-1] for x in z0], 6)
    c = oracle.step(p, [x[::-1, :] for x in z0], 6)
    for x, y, zz in zip(a, b, c):
        assert np.array_equal(x[:, ::-1], y)
        assert np.array_equal(x[::-1, :], zz)


def test_aniso_reflection_symmetry():
    """theta0 = -theta1 makes the problem symmetric under x -> L - x."""
    p = prob(model="diffusion", stencil="lap9_aniso", scheme="rk4", nx=15, ny=8, dx=0.025,
             dt=0.05, D_par=0.001171, D_perp=0.001171 / 4, theta0=-1.0, theta1=1.0)
    u = ri.diffusion_ic(15, 8, 9)
    a = oracle.step(p, u, 20)[0]
    b = oracle.step(p, [u[0][:, ::-1]], 20)[0]
    assert np.max(np.abs(a[:, ::-1] - b)) <= 1e-14


def test_crop_matches_full_domain_inside_light_cone():
    """A window cut from a larger domain evolves like the full domain at cells
    farther from the window edge than the stencil reach of the steps taken."""
    w = ri.workload("bocf_2048_aniso_rk4", nx=40, ny=30)
    par = ri.params_array("bocf")
    p = oracle.Problem.from_workload(w, params=par)
    z0 = ri.random_fields("bocf", 40, 30, 8)
    steps = 2
    full = oracle.step(p, z0, steps)
    x0, y0, wx, wy = 11, 6, 20, 18
    pc = oracle.Problem.from_workload(dict(w, nx=wx, ny=wy), params=par, x0=x0, nx_total=40)
    crop = oracle.step(pc, [a[y0:y0 + wy, x0:x0 + wx] for a in z0], steps)
    r = 4 * steps + 1
    for a, b in zip(full, crop):
        assert np.array_equal(a[y0 + r:y0 + wy - r, x0 + r:x0 + wx - r], b[r:-r, r:-r])


def test_inputs_are_seeded_and_in_range():
    a = ri.fk_ic(64, 48, 2)
    b = ri.fk_ic(64, 48, 2)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    u, v = ri.barkley_ic(32, 32, 1)
    assert u.min() >= 0.0 and u.max() <= 1.0 and v.max() < 0.5 + 1e-3
    d = ri.direction(3, 10, 10, 4)
    assert abs(sum(float(np.sum(x * x)) for x in d) - 1.0) < 1e-14
    s = ri.bocf_ic(64, 64, 3)
    assert len(s) == 4 and s[0].max() <= 1.0 + 1e-4
    f = ri.fhn_ic(40, 30, 6)
    assert np.array_equal(f[0], ri.fhn_ic(40, 30, 6)[0]) and f[0].max() <= 1.0 + 1e-3 and f[1].min() >= -0.5


# ---------------------------------------------------------------------------
# Periodic boundaries (the alternative of Sect. 3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("stencil", ["lap5", "lap9"])
@pytest.mark.parametrize("mn", [(1, 0), (0, 2), (3, 1), (5, 4)])
def test_periodic_fourier_modes_are_eigenvectors(stencil, mn):
    nx, ny, dx, D = 12, 10, 0.4, 0.7
    m, n = mn
    a, b = 2 * math.pi * m / nx, 2 * math.pi * n / ny
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    phi = np.cos(a * i + 0.3) * np.cos(b * j - 0.2)
    c = D / dx ** 2
    if stencil == "lap5":
        lam = c * ((2 * math.cos(a) - 2) + (2 * math.cos(b) - 2))
    else:
        lam = c * ((2 / 3) * (2 * math.cos(a) + 2 * math.cos(b) - 4) + (1 / 6) * (4 * math.cos(a) * math.cos(b) - 4))
    lap = oracle.laplacian(prob(stencil=stencil, nx=nx, ny=ny, dx=dx, D_par=D, bc="periodic"), phi)
    assert np.max(np.abs(lap - lam * phi)) <= 1e-13 * max(abs(lam), c)


@pytest.mark.parametrize("ab", [(1, 0), (0, 1), (2, 3), (5, 1)])
def test_periodic_flux_form_plane_wave_eigenvalue(ab):
    """Constant fibre angle: the periodic flux form maps the plane wave
    e^{i(a i + b j)} to lambda times itself, lambda from the face fluxes in
    closed form."""
    nx, ny, dx = 12, 8, 0.3
    th, dpar, dperp = 0.6, 1.3, 0.4
    a, b = 2 * math.pi * ab[0] / nx, 2 * math.pi * ab[1] / ny
    p = prob(stencil="lap9_aniso", nx=nx, ny=ny, dx=dx, D_par=dpar, D_perp=dperp, theta0=th, theta1=th,
             bc="periodic")
    dd = dpar - dperp
    dxx, dxy, dyy = dperp + dd * math.cos(th) ** 2, dd * math.cos(th) * math.sin(th), dperp + dd * math.sin(th) ** 2
    q = dxy / 4
    ea, eb = np.exp(1j * a), np.exp(1j * b)
    lam = ((dxx * (ea - 1) + q * (ea + 1) * (eb - 1 / eb)) * (1 - 1 / ea)
           + (q * (ea - 1 / ea) * (eb + 1) + dyy * (eb - 1)) * (1 - 1 / eb)) / dx ** 2
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    u = np.exp(1j * (a * i + b * j))
    out = oracle.laplacian(p, u)
    assert np.max(np.abs(out - lam * u)) <= 1e-12 * max(abs(lam), 1.0 / dx ** 2)


@pytest.mark.parametrize("stencil", ["lap5", "lap9", "lap9_aniso"])
def test_periodic_conserves_sum_and_commutes_with_shifts(stencil):
    nx, ny = 11, 9
    p = prob(stencil=stencil, scheme="rk4", nx=nx, ny=ny, dx=0.5, dt=0.01, D_par=1.0, D_perp=0.3,
             theta0=0.4, theta1=0.4, bc="periodic")
    u = np.random.default_rng(5).random((ny, nx))
    out = oracle.step(p, [u], 50)[0]
    assert abs(out.sum() - u.sum()) <= 1e-13 * u.sum()
    shifted = oracle.step(p, [np.roll(np.roll(u, 3, axis=1), -2, axis=0)], 50)[0]
    assert np.allclose(shifted, np.roll(np.roll(out, 3, axis=1), -2, axis=0), rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# Brute force and precision floor
# ---------------------------------------------------------------------------

def _brute_flux_div(p, a, j, i, rel):
    """div(rel D grad u) at cell (i, j) of the list-of-rows field a, face by
    face (Sect. 3 flux form): each of the four face fluxes from its own
    formula, zero on a boundary face, the cross-derivative terms reading
    ghost values by the half-sample mirror (index clamped into the grid) or
    the periodic wrap.  The tensor is D = D_perp I + (D_par - D_perp) f f^T
    with f = (cos t, sin t), t linear in x: at the x-face between columns k
    and k + 1, t = theta0 + (theta1 - theta0)(k + 1)/nx; at the centre of
    column k, t = theta0 + (theta1 - theta0)(k + 1/2)/nx."""
    ny, nx = p.ny, p.nx
    periodic = p.bc == "periodic"
    dd = p.D_par - p.d_perp

    def g(jj, ii):
        if periodic:
            return a[jj % ny][ii % nx]
        return a[min(max(jj, 0), ny - 1)][min(max(ii, 0), nx - 1)]

    def theta(x):
        return p.theta0 + (p.theta1 - p.theta0) * x / nx

    def xface(k):  # flux through the face between columns k and k + 1, row j
        if not periodic and (k < 0 or k >= nx - 1):
            return 0.0
        t = theta((k % nx if periodic else k) + 1.0)
        dxx = p.d_perp + dd * math.cos(t) ** 2
        dxy = dd * math.cos(t) * math.sin(t)
        du_dx = g(j, k + 1) - g(j, k)
        du_dy = ((g(j + 1, k + 1) + g(j + 1, k)) - (g(j - 1, k + 1) + g(j - 1, k))) / 4.0
        return dxx * du_dx + dxy * du_dy

    def yface(m):  # flux through the face between rows m and m + 1, column i
        if not periodic and (m < 0 or m >= ny - 1):
            return 0.0
        t = theta(i + 0.5)
        dxy = dd * math.cos(t) * math.sin(t)
        dyy = p.d_perp + dd * math.sin(t) ** 2
        du_dx = ((g(m + 1, i + 1) + g(m, i + 1)) - (g(m + 1, i - 1) + g(m, i - 1))) / 4.0
        du_dy = g(m + 1, i) - g(m, i)
        return dxy * du_dx + dyy * du_dy

    return ((xface(i) - xface(i - 1)) + (yface(j) - yface(j - 1))) * rel / (p.dx * p.dx)


@pytest.mark.parametrize("bc", ["noflux", "periodic"])
@pytest.mark.parametrize("nx,ny", [(5, 4), (1, 3), (3, 1), (2, 2), (6, 7), (1, 1)])
def test_flux_form_brute_force_face_by_face(nx, ny, bc):
    """The vectorised anisotropic flux form against scalar face-by-face
    loops on tiny grids, every cell including edges and corners, where the
    cross terms read mirrored ghosts and the boundary faces carry no flux."""
    rng = np.random.default_rng(nx * 31 + ny + (7 if bc == "periodic" else 0))
    for rep in range(3):
        th0, th1 = rng.uniform(-1.5, 1.5, 2)
        p = oracle.Problem(model="diffusion", scheme="euler", stencil="lap9_aniso", nx=nx, ny=ny, dx=0.3,
                           dt=0.01, D_par=1.3, D_perp=0.2 + 0.3 * rep, theta0=th0, theta1=th1, bc=bc)
        u = rng.standard_normal((ny, nx))
        rel = 1.0 if rep < 2 else 1.5
        got = oracle.lap_aniso(u, p, rel)
        a = u.tolist()
        ref = np.array([[_brute_flux_div(p, a, j, i, rel) for i in range(nx)] for j in range(ny)])
        scale = np.max(np.abs(u)) * 1.5 * 1.3 / 0.09
        assert np.max(np.abs(got - ref)) <= 1e-14 * scale, (rep, np.max(np.abs(got - ref)))


def test_flux_form_brute_force_detects_a_dropped_cross_term():
    """The face-by-face loops tell the flux form from a variant without the
    cross-derivative terms at the boundary (a plausible mistake: ghosts
    ignored), so the pin above is not vacuous."""
    p = oracle.Problem(model="diffusion", scheme="euler", stencil="lap9_aniso", nx=5, ny=4, dx=0.3, dt=0.01,
                       D_par=1.3, D_perp=0.2, theta0=-0.7, theta1=0.9)
    u = np.random.default_rng(5).standard_normal((4, 5))
    a = u.tolist()
    ref = np.array([[_brute_flux_div(p, a, j, i, 1.0) for i in range(5)] for j in range(4)])
    iso = oracle.Problem(model="diffusion", scheme="euler", stencil="lap9_aniso", nx=5, ny=4, dx=0.3, dt=0.01,
                         D_par=1.3, D_perp=1.3, theta0=-0.7, theta1=0.9)
    assert np.max(np.abs(oracle.lap_aniso(u, iso) - ref)) > 1e-2
    assert np.max(np.abs(oracle.lap_aniso(u, p) - ref)) <= 1e-12


def _brute_step(p, z, nsteps):
    """The explicit schemes of Sect. 3 as scalar loops over a tiny grid: the
    ghost rule of Fig. 1 (or the periodic wrap) by explicit index
    arithmetic, the 5-point or Eq. (6) 9-point sums neighbour by neighbour,
    and the reaction evaluated one cell at a time."""
    ny, nx = p.ny, p.nx
    periodic = p.bc == "periodic"
    diff = [(0, 1.0)] + ([(1, p.params[0])] if p.model == "fhn" else [])

    def at(a, j, i):
        if periodic:
            return a[j % ny][i % nx]
        return a[min(max(j, 0), ny - 1)][min(max(i, 0), nx - 1)]

    def lap(a, j, i, c):
        if p.stencil == "lap9_aniso":
            return _brute_flux_div(p, a, j, i, c * p.dx * p.dx / p.D_par)
        axial = at(a, j, i - 1) + at(a, j, i + 1) + at(a, j - 1, i) + at(a, j + 1, i) - 4.0 * a[j][i]
        if p.stencil == "lap5":
            return c * axial
        diag = at(a, j - 1, i - 1) + at(a, j - 1, i + 1) + at(a, j + 1, i - 1) + at(a, j + 1, i + 1) - 4.0 * a[j][i]
        return c * (2.0 / 3.0 * axial + 1.0 / 6.0 * diag)

    def f(y):
        nv = len(y)
        out = [[[0.0] * nx for _ in range(ny)] for _ in range(nv)]
        for j in range(ny):
            for i in range(nx):
                cell = oracle.reaction(p, [np.array([[y[m][j][i]]]) for m in range(nv)])
                for m in range(nv):
                    out[m][j][i] = float(cell[m][0, 0])
                for m, rel in diff:
                    out[m][j][i] += lap(y[m], j, i, p.D_par * rel / (p.dx * p.dx))
        return out

    def axpy(y, a, k):
        return [[[y[m][j][i] + a * k[m][j][i] for i in range(nx)] for j in range(ny)] for m in range(len(y))]

    y = [[[float(v) for v in row] for row in a] for a in z]
    dt = p.dt
    for _ in range(nsteps):
        if p.scheme == "euler":
            y = axpy(y, dt, f(y))
        elif p.scheme == "heun":
            k1 = f(y)
            k2 = f(axpy(y, dt, k1))
            y = [[[y[m][j][i] + dt / 2 * (k1[m][j][i] + k2[m][j][i]) for i in range(nx)] for j in range(ny)]
                 for m in range(len(y))]
        else:
            k1 = f(y)
            k2 = f(axpy(y, dt / 2, k1))
            k3 = f(axpy(y, dt / 2, k2))
            k4 = f(axpy(y, dt, k3))
            y = [[[y[m][j][i] + dt / 6 * (k1[m][j][i] + 2 * k2[m][j][i] + 2 * k3[m][j][i] + k4[m][j][i])
                   for i in range(nx)] for j in range(ny)] for m in range(len(y))]
    return [np.array(a) for a in y]


@pytest.mark.parametrize("model", ["diffusion", "barkley", "fk", "bocf", "fhn"])
@pytest.mark.parametrize("stencil", ["lap5", "lap9", "lap9_aniso"])
@pytest.mark.parametrize("scheme", ["euler", "heun", "rk4"])
@pytest.mark.parametrize("bc", ["noflux", "periodic"])
def test_brute_force_scalar_loops_all_models(model, stencil, scheme, bc):
    """The vectorised oracle agrees with scalar loops on a 5 x 4 grid, three
    steps, to rounding (the loops sum in their own order); the flux form with
    a rotating fibre field, face by face."""
    base = {"diffusion": "fk_1024_rk4", "barkley": "barkley_1024_rk4_adjoint", "fk": "fk_1024_rk4",
            "bocf": "bocf_2048_aniso_rk4", "fhn": "fhn_256_rk4"}[model]
    aniso = stencil == "lap9_aniso"
    w = ri.workload(base, model=model, stencil=stencil, scheme=scheme, nx=5, ny=4, bc=bc)
    w.update(D_perp=0.3 * w["D_par"] if aniso else None, theta0=-0.8 if aniso else 0.0,
             theta1=1.1 if aniso else 0.0)
    p = oracle.Problem.from_workload(w, params=ri.params_array(model))
    z = ri.random_fields(model, 5, 4, 11)
    got = oracle.step(p, z, 3)
    ref = _brute_step(p, z, 3)
    for a, b in zip(got, ref):
        assert np.max(np.abs(a - b)) <= 1e-13 * max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("model,name,n", [("fk", "fk_1024_rk4", 40), ("bocf", "bocf_2048_aniso_rk4", 36),
                                          ("barkley", "barkley_1024_rk4_adjoint", 40)])
def test_one_ulp_perturbation_floor_over_1000_steps(model, name, n):
    """How far FP64 rounding differences can grow: two oracle runs of 1000
    steps from initial states one ulp apart stay within 1e-12 (relative
    L-infinity), below the 1e-11 parity gate, for the steep-front models."""
    w = ri.workload(name, nx=n, ny=n)
    p = oracle.Problem.from_workload(w, params=ri.params_array(model))
    z0 = ri.initial_condition(w) if model != "bocf" else ri.bocf_ic(n, n, 3, amp=1e-2)
    a = oracle.step(p, z0, 1000)
    b = oracle.step(p, [np.nextafter(x, np.inf) for x in z0], 1000)
    err = max(float(np.max(np.abs(x - y)) / np.max(np.abs(y))) for x, y in zip(a, b))
    assert err <= 1e-12, err


@pytest.mark.parametrize("case", conditioning.CASES, ids=lambda c: "-".join(map(str, c[:4])))
def test_rounding_floor_of_the_long_horizon_gradient_cases(case):
    """The cases the GPU gradient is held to 1e-11 of the oracle's over 200
    RK4 steps are well conditioned: one-ulp random perturbations after every
    step move the oracle's state by at most 1e-13 over the horizon (measured
    7e-15 .. 1.2e-14), and its gradient of L = dx^2 sum u(T)^2 moves by at
    most 1e-13 when the initial state moves by one ulp at random and dt by one
    ulp (every step perturbed)."""
    model, stencil, nx, ny, ic = case
    w = conditioning.workload(model, stencil, nx, ny)
    p = oracle.Problem.from_workload(w, params=ri.params_array(model))
    z0 = conditioning.initial(model, nx, ny, ic)
    assert conditioning.state_floor(p, z0) <= 1e-13
    steps = conditioning.STEPS
    zT = oracle.step(p, z0, steps)
    lam = [2.0 * p.dx ** 2 * zT[0]] + [np.zeros_like(a) for a in zT[1:]]
    g0 = oracle.vjp(p, z0, lam, steps, checkpoint_every=conditioning.EVERY)
    rng = np.random.default_rng(2)
    z1 = [np.where(rng.random(a.shape) < 0.5, np.nextafter(a, np.inf), np.nextafter(a, -np.inf)) for a in z0]
    p1 = dataclasses.replace(p, dt=float(np.nextafter(p.dt, np.inf)))
    g1 = oracle.vjp(p1, z1, lam, steps, checkpoint_every=conditioning.EVERY)
    err = max(float(np.max(np.abs(x - y)) / np.max(np.abs(y))) for x, y in zip(g1, g0))
    assert 0.0 < err <= 1e-13, err


def test_barkley_spiral_seed_is_ill_conditioned_while_the_spiral_forms():
    """Why the Barkley spiral seed is not a case of the 1e-11 gradient test:
    on an 80 x 72 grid, one-ulp random perturbations after every RK4 step grow
    to more than 1e-5 of the state within 200 steps (measured 4e-3), so two
    correct implementations that round differently disagree by that much."""
    w = conditioning.workload("barkley", "lap9", 80, 72)
    p = oracle.Problem.from_workload(w, params=ri.params_array("barkley"))
    assert conditioning.state_floor(p, conditioning.initial("barkley", 80, 72, "spiral")) >= 1e-5


def test_fhn_rk4_precision_floor_saturates():
    """Sect. 5 after Table 1: for FitzHugh-Nagumo the relative error of RK4
    falls at fourth order as dt shrinks until it saturates at the FP64
    rounding floor (the paper: around 1e-14).  Richardson differences of
    successive dt halvings (16^2, dx = 0.04, 9-point, T = 0.004) show order 4
    down to ~1e-14 and then stop falling at ~1e-15."""
    w = ri.workload("fhn_256_rk4", nx=16, ny=16)
    z0 = ri.initial_condition(w)
    sols = []
    for lv in range(10):
        dt = 2e-4 / 2 ** lv
        p = oracle.Problem.from_workload(dict(w, dt=dt), params=ri.params_array("fhn"))
        sols.append(np.concatenate([a.ravel() for a in oracle.step(p, z0, int(round(0.004 / dt)))]))
    e = [float(np.linalg.norm(sols[k] - sols[k + 1]) / np.linalg.norm(sols[k + 1])) for k in range(9)]
    orders = [math.log2(e[k] / e[k + 1]) for k in range(8)]
    assert all(abs(o - 4.0) < 0.2 for o in orders[:6]), orders
    assert 1e-16 < min(e) < 1e-14, e          # the floor is reached ...
    assert e[-1] > 0.5 * e[-2], e              # ... and the error stops falling there


def test_fp64_floor_against_long_double():
    """The same FitzHugh-Nagumo run (16 x 16, 9-point, RK4, 200 steps) in
    FP64 and in extended precision differ by no more than the FP64
    rounding floor."""
    assert np.finfo(np.longdouble).eps < np.finfo(np.float64).eps
    w = ri.workload("fhn_256_rk4", nx=16, ny=16)
    p = oracle.Problem.from_workload(w, params=ri.params_array("fhn"))
    z0 = ri.random_fields("fhn", 16, 16, 4)
    a = oracle.step(p, z0, 200)
    b = oracle.step(p, [x.astype(np.longdouble) for x in z0], 200)
    assert b[0].dtype == np.longdouble
    err = max(float(np.max(np.abs(x - y)) / np.max(np.abs(y))) for x, y in zip(a, b))
    assert 0.0 < err <= 1e-13, err


@pytest.mark.parametrize("model", ["fk", "bocf"])
@pytest.mark.parametrize("stencil", ["lap5", "lap9", "lap9_aniso"])
@pytest.mark.parametrize("scheme", ["rush_larsen", "implicit_euler"])
def test_gate_scheme_adjoint_dot_product(model, stencil, scheme):
    """The gate steps' adjoint against the complex-step tangent of the whole
    flow (an independent derivative): <J v, w> = <v, J^T w>."""
    p, z0 = case_problem(model, stencil, scheme)
    nv = len(z0)
    v = ri.direction(nv, p.nx, p.ny, 31)
    w = ri.direction(nv, p.nx, p.ny, 32)
    _, jv = oracle.jvp(p, z0, v, 9)
    jtw = oracle.vjp(p, z0, w, 9, checkpoint_every=4)
    a = float(flat(jv) @ flat(w))
    b = float(flat(v) @ flat(jtw))
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


@pytest.mark.parametrize("model,stencil,scheme", [("fk", "lap9", "rush_larsen"), ("bocf", "lap5", "implicit_euler")])
def test_gate_scheme_vjp_equals_transpose_of_dense_jacobian(model, stencil, scheme):
    p, z0 = case_problem(model, stencil, scheme, nx=4, ny=3)
    nv, n = len(z0), 12
    J = np.zeros((nv * n, nv * n))
    for k in range(nv * n):
        e = np.zeros(nv * n)
        e[k] = 1.0
        _, jv = oracle.jvp(p, z0, [a.reshape(3, 4) for a in np.split(e, nv)], 3)
        J[:, k] = flat(jv)
    lam = ri.direction(nv, 4, 3, 5)
    got = flat(oracle.vjp(p, z0, lam, 3, checkpoint_every=2))
    assert np.max(np.abs(got - J.T @ flat(lam))) <= 1e-13 * np.max(np.abs(J.T @ flat(lam)))
