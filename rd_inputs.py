"""Seeded synthetic inputs for the 2-D cardiac reaction-diffusion workloads.

This module is shared by the oracle-based tests, the GPU tests and the
benchmark.  It holds only data and random-number draws: model parameter
sets (in the order the C ABI documents), workload descriptions, initial
conditions and perturbation directions.  It contains none of the method's
arithmetic -- no stencil, reaction, Jacobian or time-stepping code -- so
that the oracle and the HIP path remain independent of each other.

Models (Marcotte & Grigoriev, Sect. 2):
  * ``barkley``   -- 2-variable Barkley excitable medium (u diffusive).
  * ``fk``        -- 3-variable Fenton-Karma model (u, v, w).
  * ``bocf``      -- 4-variable Bueno-Orovio-Cherry-Fenton model, Eq. (5).
  * ``diffusion`` -- pure diffusion of one field (N = 0), a test model.

All random numbers come from ``numpy.random.default_rng(seed)`` (PCG64).
Arrays are float64, shape ``(ny, nx)``, x (column index i) fastest.
"""
from __future__ import annotations

import math

import numpy as np

# ----------------------------------------------------------------------------
# Parameter sets.  The order of each tuple is the order of the ``params``
# array passed through the C ABI and to the oracle.
# ----------------------------------------------------------------------------

BARKLEY_PARAM_NAMES = ("a", "b", "eps")
BARKLEY_PARAMS = {"a": 0.75, "b": 0.02, "eps": 0.02}

# FitzHugh-Nagumo, Eq. (3), with the nondimensional values of Sect. 2:
# (delta, eps, a1, a0) = (1.5, 0.05, 1.5, -0.1), dx = dy = 0.04.
FHN_PARAM_NAMES = ("delta", "eps", "a1", "a0")
FHN_PARAMS = {"delta": 1.5, "eps": 0.05, "a1": 1.5, "a0": -0.1}

# Fenton & Karma (1998), parameter set fitted to the Beeler-Reuter model.
# Times in ms, voltage dimensionless.
FK_PARAM_NAMES = (
    "tau_v_plus", "tau_v1_minus", "tau_v2_minus", "tau_w_plus", "tau_w_minus",
    "tau_d", "tau_0", "tau_r", "tau_si", "k_si", "u_c_si", "u_c", "u_v",
)
FK_PARAMS = {
    "tau_v_plus": 3.33, "tau_v1_minus": 19.6, "tau_v2_minus": 1000.0,
    "tau_w_plus": 667.0, "tau_w_minus": 11.0, "tau_d": 0.25, "tau_0": 8.3,
    "tau_r": 50.0, "tau_si": 45.0, "k_si": 10.0, "u_c_si": 0.85,
    "u_c": 0.13, "u_v": 0.055,
}

# Bueno-Orovio, Cherry & Fenton (2008), epicardial parameter set.
BOCF_PARAM_NAMES = (
    "u_o", "u_u", "theta_v", "theta_w", "theta_v_minus", "theta_o",
    "tau_v1_minus", "tau_v2_minus", "tau_v_plus",
    "tau_w1_minus", "tau_w2_minus", "k_w_minus", "u_w_minus", "tau_w_plus",
    "tau_fi", "tau_o1", "tau_o2",
    "tau_so1", "tau_so2", "k_so", "u_so",
    "tau_s1", "tau_s2", "k_s", "u_s",
    "tau_si", "tau_w_inf", "w_inf_star",
)
BOCF_PARAMS = {
    "u_o": 0.0, "u_u": 1.55, "theta_v": 0.3, "theta_w": 0.13,
    "theta_v_minus": 0.006, "theta_o": 0.006,
    "tau_v1_minus": 60.0, "tau_v2_minus": 1150.0, "tau_v_plus": 1.4506,
    "tau_w1_minus": 60.0, "tau_w2_minus": 15.0, "k_w_minus": 65.0,
    "u_w_minus": 0.03, "tau_w_plus": 200.0,
    "tau_fi": 0.11, "tau_o1": 400.0, "tau_o2": 6.0,
    "tau_so1": 30.0181, "tau_so2": 0.9957, "k_so": 2.0458, "u_so": 0.65,
    "tau_s1": 2.7342, "tau_s2": 16.0, "k_s": 2.0994, "u_s": 0.9087,
    "tau_si": 1.8875, "tau_w_inf": 0.07, "w_inf_star": 0.94,
}

PARAM_NAMES = {
    "diffusion": (),
    "barkley": BARKLEY_PARAM_NAMES,
    "fk": FK_PARAM_NAMES,
    "bocf": BOCF_PARAM_NAMES,
    "fhn": FHN_PARAM_NAMES,
}
DEFAULT_PARAMS = {
    "diffusion": {},
    "barkley": BARKLEY_PARAMS,
    "fk": FK_PARAMS,
    "bocf": BOCF_PARAMS,
    "fhn": FHN_PARAMS,
}
N_FIELDS = {"diffusion": 1, "barkley": 2, "fk": 3, "bocf": 4, "fhn": 2}

# Width parameter of the smoothed step function (Sect. 2): k = 28.4.
STEP_K = 28.4


def params_array(model: str, overrides: dict | None = None) -> np.ndarray:
    """Parameter vector of ``model`` in ABI order, with optional overrides."""
    vals = dict(DEFAULT_PARAMS[model])
    if overrides:
        unknown = set(overrides) - set(vals)
        if unknown:
            raise KeyError(f"unknown {model} parameters: {sorted(unknown)}")
        vals.update(overrides)
    return np.array([vals[n] for n in PARAM_NAMES[model]], dtype=np.float64)


# ----------------------------------------------------------------------------
# Workloads.  Each is a plain dict; both the oracle's and the binding's
# problem descriptions are built from it by the caller.
# ----------------------------------------------------------------------------

def workload(name: str, **overrides) -> dict:
    """Named workload (problem description + initial-condition recipe)."""
    w = dict(_WORKLOADS[name])
    w.update(overrides)
    return w


_BASE = dict(D_perp=None, theta0=0.0, theta1=0.0, step_k=STEP_K, checkpoint_every=0, bc="noflux", nz=1)

_WORKLOADS = {
    # Barkley 128x128, 5-point Laplacian, forward Euler, 1000 steps.
    "barkley_128_euler": dict(_BASE, model="barkley", stencil="lap5", scheme="euler",
                              nx=128, ny=128, dx=0.5, dt=0.02, nsteps=1000,
                              D_par=1.0, ic="barkley", seed=1),
    # Fenton-Karma 1024x1024, isotropic 9-point Laplacian, RK4, 10000 steps.
    "fk_1024_rk4": dict(_BASE, model="fk", stencil="lap9", scheme="rk4",
                        nx=1024, ny=1024, dx=0.025, dt=0.1, nsteps=10000,
                        D_par=0.001, ic="fk", seed=2),
    # Bueno-Orovio 2048x2048, anisotropic flux-form 9-point stencil with
    # fibre angle rotating linearly from -60 to +60 degrees across x, RK4.
    "bocf_2048_aniso_rk4": dict(_BASE, model="bocf", stencil="lap9_aniso", scheme="rk4",
                                nx=2048, ny=2048, dx=0.025, dt=0.05, nsteps=5000,
                                D_par=0.001171, D_perp=0.001171 / 4.0,
                                theta0=-math.pi / 3.0, theta1=math.pi / 3.0,
                                ic="bocf", seed=3),
    # Barkley 1024x1024 RK4 4000 steps (adjoint workload), checkpoints every 64.
    # FitzHugh-Nagumo 256x256 (the grid of the convergence study, Sect. 5),
    # dx = 0.04, 9-point Laplacian on u and v (v with delta D), RK4; dt inside
    # every scheme's stability limit for both stencils.
    "fhn_256_rk4": dict(_BASE, model="fhn", stencil="lap9", scheme="rk4",
                        nx=256, ny=256, dx=0.04, dt=2e-4, nsteps=1000,
                        D_par=1.0, ic="fhn", seed=6),
    "barkley_1024_rk4_adjoint": dict(_BASE, model="barkley", stencil="lap5", scheme="rk4",
                                     nx=1024, ny=1024, dx=0.5, dt=0.02, nsteps=4000,
                                     D_par=1.0, ic="barkley", seed=5,
                                     checkpoint_every=64),
    # Fenton-Karma on a 256^3 block (3-D tissue, which the conclusion looks
    # ahead to), compact 27-point operator, RK4; the 2-D workload's spacing
    # and step, a scroll-wave seed (the broken-wave seed extruded along z).
    "fk_256cube_lap27_rk4": dict(_BASE, model="fk", stencil="lap27", scheme="rk4",
                                 nx=256, ny=256, nz=256, dx=0.025, dt=0.1, nsteps=1000,
                                 D_par=0.001, ic="fk3d", seed=7),
}

# Ensemble of Fenton-Karma instances on uneven grids, tangent-linear run:
# 16 instances each of 256^2, 384^2, 512^2 and 768^2, 2000 RK4 steps.
FK_BATCH_SIZES = (256, 384, 512, 768)
FK_BATCH_PER_SIZE = 16


def fk_batch_workloads(nsteps: int = 2000, sizes=FK_BATCH_SIZES,
                       per_size: int = FK_BATCH_PER_SIZE) -> list[dict]:
    out = []
    r = 0
    for n in sizes:
        for _ in range(per_size):
            out.append(workload("fk_1024_rk4", nx=n, ny=n, nsteps=nsteps,
                                seed=4000 + r, direction_seed=4100 + r))
            r += 1
    return out


# ----------------------------------------------------------------------------
# Initial conditions (uniform noise U[0, amp) added per field in model order).
# ----------------------------------------------------------------------------

def _noise(rng, fields, amp):
    for f in fields:
        f += rng.random(f.shape) * amp
    return fields


def barkley_ic(nx: int, ny: int, seed: int, amp: float = 1e-3) -> list[np.ndarray]:
    """Cross-field spiral seed: u = 1 for x < L/2, v = 0.5 for y < L/2.

    The noise U[0, amp) points into the model's range u in [0, 1]: it is
    subtracted where u = 1 and added where u = 0.  (u = 1 is an invariant
    line of the Barkley reaction; a state above it runs away once
    v > a - b, so noise added on top of u = 1 would leave the model.)
    """
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    excited = np.broadcast_to(i < nx / 2, (ny, nx))
    v = np.ascontiguousarray(np.where(j < ny / 2, 0.5, 0.0) * np.ones((1, nx)))
    rng = np.random.default_rng(seed)
    nu = rng.random((ny, nx)) * amp
    u = np.where(excited, 1.0 - nu, nu)
    v += rng.random((ny, nx)) * amp
    return [np.ascontiguousarray(u), v]


def _fk_pattern(nx: int, ny: int):
    """Broken-wave seed: excited stripe on the upper-left edge, refractory
    lower-left quadrant, rest elsewhere."""
    u = np.zeros((ny, nx))
    v = np.ones((ny, nx))
    w = np.ones((ny, nx))
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    stripe = (i < max(nx // 16, 1)) & (j < ny / 2)
    quad = (i < nx / 2) & (j >= ny / 2)
    u[stripe] = 1.0
    v[quad] = 0.0
    return u, v, w, stripe, quad


def fk_ic(nx: int, ny: int, seed: int, amp: float = 1e-4) -> list[np.ndarray]:
    u, v, w, _, _ = _fk_pattern(nx, ny)
    rng = np.random.default_rng(seed)
    return _noise(rng, [u, v, w], amp)


def fk_ic3(nx: int, ny: int, nz: int, seed: int, amp: float = 1e-4) -> list[np.ndarray]:
    """Scroll-wave seed: the 2-D broken-wave seed on every plane, plus noise."""
    u, v, w, _, _ = _fk_pattern(nx, ny)
    rng = np.random.default_rng(seed)
    return _noise(rng, [np.repeat(f[None], nz, axis=0) for f in (u, v, w)], amp)


def bocf_ic(nx: int, ny: int, seed: int, amp: float = 1e-4, blocks: int = 4) -> list[np.ndarray]:
    """Multi-spiral seed: a blocks x blocks grid of broken-wave seeds, each
    rotated (square blocks) or flipped by a seeded multiple of 90 degrees."""
    rng = np.random.default_rng(seed)
    u = np.zeros((ny, nx))
    v = np.ones((ny, nx))
    w = np.ones((ny, nx))
    s = np.zeros((ny, nx))
    by_edges = np.linspace(0, ny, blocks + 1).astype(int)
    bx_edges = np.linspace(0, nx, blocks + 1).astype(int)
    for bj in range(blocks):
        for bi in range(blocks):
            y0, y1 = by_edges[bj], by_edges[bj + 1]
            x0, x1 = bx_edges[bi], bx_edges[bi + 1]
            h, wd = y1 - y0, x1 - x0
            if h == 0 or wd == 0:
                continue
            _, _, _, stripe, quad = _fk_pattern(wd, h)
            rot = int(rng.integers(4))
            if h == wd:
                stripe = np.rot90(stripe, rot)
                quad = np.rot90(quad, rot)
            else:
                if rot & 1:
                    stripe, quad = stripe[:, ::-1], quad[:, ::-1]
                if rot & 2:
                    stripe, quad = stripe[::-1, :], quad[::-1, :]
            u[y0:y1, x0:x1][stripe] = 1.0
            v[y0:y1, x0:x1][quad] = 0.0
            w[y0:y1, x0:x1][quad] = 0.0
    return _noise(rng, [u, v, w, s], amp)


def fhn_ic(nx: int, ny: int, seed: int, amp: float = 1e-3) -> list[np.ndarray]:
    """Cross-field spiral seed for Eq. (3): u = 1 for x < L/2 (else -1),
    v = 0.5 for y < L/2 (else -0.5), plus noise U[0, amp) on u then v."""
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    u = np.where(i < nx / 2, 1.0, -1.0) * np.ones((ny, 1))
    v = np.where(j < ny / 2, 0.5, -0.5) * np.ones((1, nx))
    rng = np.random.default_rng(seed)
    return _noise(rng, [np.ascontiguousarray(u), np.ascontiguousarray(v)], amp)


def diffusion_ic(nx: int, ny: int, seed: int) -> list[np.ndarray]:
    """Random field in [0, 1) for the pure-diffusion test model."""
    rng = np.random.default_rng(seed)
    return [rng.random((ny, nx))]


def initial_condition(w: dict) -> list[np.ndarray]:
    """Initial fields for workload dict ``w`` (keys ic, nx, ny, seed)."""
    kind = w["ic"]
    if kind == "barkley":
        return barkley_ic(w["nx"], w["ny"], w["seed"])
    if kind == "fk":
        return fk_ic(w["nx"], w["ny"], w["seed"])
    if kind == "fk3d":
        return fk_ic3(w["nx"], w["ny"], w["nz"], w["seed"])
    if kind == "bocf":
        return bocf_ic(w["nx"], w["ny"], w["seed"])
    if kind == "diffusion":
        return diffusion_ic(w["nx"], w["ny"], w["seed"])
    if kind == "fhn":
        return fhn_ic(w["nx"], w["ny"], w["seed"])
    raise ValueError(f"unknown initial condition {kind!r}")


def random_fields(model: str, nx: int, ny: int, seed: int, nz: int | None = None) -> list[np.ndarray]:
    """Random state inside the physiological range of ``model`` (tests);
    arrays of shape (ny, nx), or (nz, ny, nx) when nz is given."""
    rng = np.random.default_rng(seed)
    nv = N_FIELDS[model]
    shape = (ny, nx) if nz is None else (nz, ny, nx)
    if model == "fhn":  # u in (-1.2, 1.2), v in (-0.6, 0.6)
        return [(rng.random(shape) - 0.5) * 2.4, (rng.random(shape) - 0.5) * 1.2]
    hi = {"diffusion": 1.0, "barkley": 1.0, "fk": 1.0, "bocf": 1.55}[model]
    u = rng.random(shape) * hi
    return [u] + [rng.random(shape) for _ in range(nv - 1)]


def direction(nfields: int, nx: int, ny: int, seed: int, nz: int | None = None) -> list[np.ndarray]:
    """Gaussian direction over all fields, scaled to unit Euclidean norm."""
    rng = np.random.default_rng(seed)
    shape = (ny, nx) if nz is None else (nz, ny, nx)
    d = [rng.standard_normal(shape) for _ in range(nfields)]
    nrm = math.sqrt(sum(float(np.sum(a * a)) for a in d))
    return [a / nrm for a in d]
