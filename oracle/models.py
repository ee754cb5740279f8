"""Reaction terms N[z] of Eq. (1) and the smoothed step function H_k.

Marcotte & Grigoriev, Sect. 2.  Each model returns the list of pointwise
rates (N_u, N_h1, ...) for the state z = (u, h1, ...); the integrator adds
the diffusion terms to the rates of the diffusive fields (`diffusive_fields`):
the voltage u for every model, and also v for FitzHugh-Nagumo (Eq. 3), whose
second field diffuses with the relative coefficient delta.

Constant divisors (time constants) are applied as multiplications by their
reciprocals, computed once per call; divisors that depend on u (tau(u)) are
true divisions.  Parameters arrive as a flat tuple in the documented order
(see the C header and the input module).
"""
from __future__ import annotations

import numpy as np

from .problem import Problem

_NFIELDS = {"diffusion": 1, "barkley": 2, "fk": 3, "bocf": 4, "fhn": 2}
_NPARAMS = {"diffusion": 0, "barkley": 3, "fk": 13, "bocf": 28, "fhn": 4}


def n_fields(model: str) -> int:
    return _NFIELDS[model]


def n_params(model: str) -> int:
    return _NPARAMS[model]


def diffusive_fields(prob: Problem):
    """[(field index, diffusivity relative to D_par)] of the problem's model.

    Eq. (3): u diffuses with D (the nondimensional 1 of the paper, D_par
    here) and v with delta D, delta the model's first parameter.  All other
    models diffuse u alone."""
    if prob.model == "fhn":
        return [(0, 1.0), (1, float(prob.params[0]))]
    return [(0, 1.0)]


def smooth_step(x, k: float):
    """Smoothed step H_k of Sect. 2.

    0 for kx < -1/2, (3 - 2kx - 1)(kx + 1/2)^2 for |kx| <= 1/2, 1 for kx > 1/2.
    With t = kx + 1/2 the middle branch is t^2 (3 - 2t).  k = inf gives the
    sharp Heaviside function with H(0) = 1.  Branches are taken on the real
    part so that complex-step differentiation passes through.
    """
    x = np.asarray(x)
    if np.isinf(k):
        return np.where(np.real(x) >= 0.0, 1.0, 0.0).astype(x.dtype)
    t = k * x + 0.5
    tr = np.real(t)
    mid = t * t * (3.0 - 2.0 * t)
    return np.where(tr <= 0.0, 0.0, np.where(tr >= 1.0, 1.0, mid)).astype(mid.dtype)


def _barkley(z, p):
    """du = (1/eps) u (1 - u) (u - (v + b)/a),  dv = u - v."""
    u, v = z
    a, b, eps = p
    inv_a = 1.0 / a
    inv_eps = 1.0 / eps
    uth = (v + b) * inv_a
    fu = ((inv_eps * u) * (1.0 - u)) * (u - uth)
    fv = u - v
    return [fu, fv]


def _fitzhugh_nagumo(z, p):
    """Eq. (3) without its diffusion terms:
    du = u - v - u^3,  dv = eps (u - a1 v - a0);  params (delta, eps, a1, a0)."""
    u, v = z
    _delta, eps, a1, a0 = p
    fu = (u - v) - (u * u) * u
    fv = eps * ((u - a1 * v) - a0)
    return [fu, fv]


def _fenton_karma(z, p, k):
    """Three-variable Fenton-Karma model with the gates written through H_k.

    J_fi = -v p (1 - u)(u - u_c)/tau_d, J_so = u (1 - p)/tau_0 + p/tau_r,
    J_si = -w (1 + tanh(k_si (u - u_c_si)))/(2 tau_si), p = H(u - u_c),
    q = H(u - u_v), tau_v^- = q tau_v1^- + (1 - q) tau_v2^-,
    dv = (1 - p)(1 - v)/tau_v^- - p v/tau_v^+,
    dw = (1 - p)(1 - w)/tau_w^- - p w/tau_w^+.
    """
    u, v, w = z
    (tau_vp, tau_v1m, tau_v2m, tau_wp, tau_wm, tau_d, tau_0, tau_r, tau_si,
     k_si, u_csi, u_c, u_v) = p
    inv_tau_d = 1.0 / tau_d
    inv_tau_0 = 1.0 / tau_0
    inv_tau_r = 1.0 / tau_r
    inv_2tau_si = 1.0 / (2.0 * tau_si)
    inv_tau_vp = 1.0 / tau_vp
    inv_tau_wp = 1.0 / tau_wp
    inv_tau_wm = 1.0 / tau_wm
    pp = smooth_step(u - u_c, k)
    qq = smooth_step(u - u_v, k)
    j_fi = -(((v * pp) * (1.0 - u)) * (u - u_c)) * inv_tau_d
    j_so = (u * (1.0 - pp)) * inv_tau_0 + pp * inv_tau_r
    j_si = -(w * (1.0 + np.tanh(k_si * (u - u_csi)))) * inv_2tau_si
    tau_vm = qq * tau_v1m + (1.0 - qq) * tau_v2m
    fu = -((j_fi + j_so) + j_si)
    fv = ((1.0 - pp) * (1.0 - v)) / tau_vm - (pp * v) * inv_tau_vp
    fw = ((1.0 - pp) * (1.0 - w)) * inv_tau_wm - (pp * w) * inv_tau_wp
    return [fu, fv, fw]


def _bueno_orovio(z, p, k):
    """Four-variable minimal model, Eq. (5) with the currents and the
    alpha/beta gate form printed under it; tau(u), v_inf and w_inf follow
    Bueno-Orovio, Cherry & Fenton (2008).  The s equation divides by
    tau_s(u) (a rate, units 1/ms).  J_si uses the constant tau_si."""
    u, v, w, s = z
    (u_o, u_u, th_v, th_w, th_vm, th_o, tau_v1m, tau_v2m, tau_vp,
     tau_w1m, tau_w2m, k_wm, u_wm, tau_wp, tau_fi, tau_o1, tau_o2,
     tau_so1, tau_so2, k_so, u_so, tau_s1, tau_s2, k_s, u_s,
     tau_si, tau_winf, w_infstar) = p

    def H(x):
        return smooth_step(x, k)

    inv_tau_fi = 1.0 / tau_fi
    inv_tau_si = 1.0 / tau_si
    inv_tau_vp = 1.0 / tau_vp
    inv_tau_wp = 1.0 / tau_wp
    inv_tau_winf = 1.0 / tau_winf

    h_v = H(u - th_v)
    h_v_neg = H(th_v - u)
    h_w = H(u - th_w)
    h_w_neg = H(th_w - u)
    h_vm = H(u - th_vm)
    h_o = H(u - th_o)

    tau_vm = (1.0 - h_vm) * tau_v1m + h_vm * tau_v2m
    tau_wm = tau_w1m + (tau_w2m - tau_w1m) * ((1.0 + np.tanh(k_wm * (u - u_wm))) * 0.5)
    tau_so = tau_so1 + (tau_so2 - tau_so1) * ((1.0 + np.tanh(k_so * (u - u_so))) * 0.5)
    tau_s = (1.0 - h_w) * tau_s1 + h_w * tau_s2
    tau_o = (1.0 - h_o) * tau_o1 + h_o * tau_o2
    v_inf = H(th_vm - u)
    w_inf = (1.0 - h_o) * (1.0 - u * inv_tau_winf) + h_o * w_infstar

    j_fi = -(((v * h_v) * (u - th_v)) * (u_u - u)) * inv_tau_fi
    j_so = ((u - u_o) * h_w_neg) / tau_o + h_w / tau_so
    j_si = -((h_w * w) * s) * inv_tau_si
    fu = -((j_fi + j_so) + j_si)

    alpha_v = -(h_v * inv_tau_vp) - h_v_neg / tau_vm
    beta_v = (h_v_neg * v_inf) / tau_vm
    fv = alpha_v * v + beta_v
    alpha_w = -(h_w * inv_tau_wp) - h_w_neg / tau_wm
    beta_w = (h_w_neg * w_inf) / tau_wm
    fw = alpha_w * w + beta_w
    fs = ((1.0 + np.tanh(k_s * (u - u_s))) * 0.5 - s) / tau_s
    return [fu, fv, fw, fs]


def reaction(prob: Problem, z):
    """Pointwise reaction rates N[z] for the problem's model."""
    nv = n_fields(prob.model)
    if len(z) != nv:
        raise ValueError(f"{prob.model} has {nv} fields, got {len(z)}")
    if len(prob.params) != n_params(prob.model):
        raise ValueError(f"{prob.model} takes {n_params(prob.model)} parameters, "
                         f"got {len(prob.params)}")
    if prob.model == "diffusion":
        return [np.zeros_like(z[0])]
    if prob.model == "barkley":
        return _barkley(z, prob.params)
    if prob.model == "fhn":
        return _fitzhugh_nagumo(z, prob.params)
    if prob.model == "fk":
        return _fenton_karma(z, prob.params, prob.step_k)
    return _bueno_orovio(z, prob.params, prob.step_k)


def gate_fields(prob: Problem):
    """Fields whose rate is linear in the field itself, dg/dt = alpha g + beta
    with alpha, beta depending on the other fields: the gating variables of
    the gated models (Fenton-Karma v, w; Bueno-Orovio v, w, s)."""
    if prob.model in ("fk", "bocf"):
        return list(range(1, n_fields(prob.model)))
    return []


def gate_coefficients(prob: Problem, z):
    """{g: (alpha_g, beta_g)} with N_g(z) = alpha_g z_g + beta_g: beta_g is the
    rate with z_g set to 0 and alpha_g the change of the rate when z_g goes
    from 0 to 1 (exact for a rate linear in z_g)."""
    out = {}
    for g in gate_fields(prob):
        z0, z1 = list(z), list(z)
        z0[g] = np.zeros_like(z[g])
        z1[g] = np.ones_like(z[g])
        n0 = reaction(prob, z0)[g]
        n1 = reaction(prob, z1)[g]
        out[g] = (n1 - n0, n0)
    return out


COMPLEX_STEP = 1e-30


def reaction_jacobian(prob: Problem, z):
    """Pointwise Jacobian J[m][l] = dN_m/dz_l by complex-step differentiation
    of ``reaction`` (exact to rounding for these analytic rates)."""
    nv = n_fields(prob.model)
    jac = [[None] * nv for _ in range(nv)]
    base = [np.asarray(a, dtype=np.complex128) for a in z]
    for l in range(nv):
        pert = list(base)
        pert[l] = base[l] + 1j * COMPLEX_STEP
        out = reaction(prob, pert)
        for m in range(nv):
            jac[m][l] = np.imag(out[m]) / COMPLEX_STEP
    return jac
