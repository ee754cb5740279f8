"""Explicit time integration of Eq. (1), its tangent-linear map and adjoint.

Marcotte & Grigoriev, Sect. 3 and Sect. 4: every explicit scheme is a
sequence of stages, each of which evaluates the non-local diffusion term,
then the local reaction terms, and combines them in an Euler-like update.

  Euler : z' = z + dt k1
  Heun  : k1 = f(z), k2 = f(z + dt k1),                z' = z + (dt/2)(k1 + k2)
  RK4   : k1 = f(z), k2 = f(z + (dt/2) k1), k3 = f(z + (dt/2) k2),
          k4 = f(z + dt k3),                           z' = z + (dt/6)(k1 + 2 k2 + 2 k3 + k4)

with f(z) = (L u + N_u(z), N_h(z)): only the voltage u diffuses, except in
FitzHugh-Nagumo (Eq. 3), where v diffuses too, with the operator scaled by
delta.

Rush-Larsen and implicit Euler (Sect. 3; Table 1 applies them to the
Bueno-Orovio model only, and only to its non-diffusive variables): the
voltage takes an explicit Euler step; each gate g, whose rate is alpha g +
beta with alpha, beta frozen at z_n, takes the exponential step
  g' = g e^{alpha dt} + (beta / alpha)(e^{alpha dt} - 1)        (Rush-Larsen)
or the implicit Euler step of that linear equation
  g' = (g + dt beta) / (1 - dt alpha)                           (implicit Euler).

Tangent-linear map: the exact derivative of the discrete flow, obtained by
running the same forward code in complex arithmetic from z + i h dz and
reading Im / h (complex-step differentiation; no subtraction, so exact to
rounding for these analytic operations).

Adjoint: the exact transpose of the discrete step, stage by stage in
reverse order.  For stage inputs Y_s = z + sum_j A_sj k_j and output
z' = z + sum_s B_s k_s:  zbar = lam, kbar_s = B_s lam, then for s from the
last stage down to the first, Ybar_s = J(Y_s)^T kbar_s, zbar += Ybar_s and
kbar_j += A_sj Ybar_s (j < s).  J(Y)^T a = (L^T a_u + sum_m dN_m/du a_m,
sum_m dN_m/dh a_m), with L^T the transposed sparse operator and the
pointwise Jacobian from complex-step differentiation of the reaction.
A gate step is transposed as its pointwise part (complex-step columns of the
voltage's reaction update and of each gate update) plus dt L^T on the
diffusive field.
"""
from __future__ import annotations

import numpy as np

from .models import diffusive_fields, gate_coefficients, gate_fields, n_fields, reaction, reaction_jacobian
from .problem import Problem
from .stencils import laplacian, laplacian_matrix


def rhs(prob: Problem, z):
    """f(z): diffusion on the diffusive fields plus the pointwise reaction."""
    n = list(reaction(prob, z))
    for f, rel in diffusive_fields(prob):
        n[f] = laplacian(prob, z[f], rel) + n[f]
    return n


def transposed_operators(prob: Problem):
    """{field: L_f^T} for the diffusive fields (sparse)."""
    return {f: laplacian_matrix(prob, rel).T.tocsr() for f, rel in diffusive_fields(prob)}


def _axpy(z, a, k):
    return [zi + a * ki for zi, ki in zip(z, k)]


def _coefficients(prob: Problem):
    """(A, B) of the scheme with the constants exactly as the forward uses them."""
    dt = prob.dt
    if prob.scheme in ("rush_larsen", "implicit_euler"):
        raise ValueError(f"{prob.scheme} is not a Runge-Kutta scheme (no stage coefficients)")
    if prob.scheme == "euler":
        return [[]], [dt]
    if prob.scheme == "heun":
        h2 = dt * 0.5
        return [[], [dt]], [h2, h2]
    h2 = dt * 0.5
    h6 = dt / 6.0
    return [[], [h2], [0.0, h2], [0.0, 0.0, dt]], [h6, 2.0 * h6, 2.0 * h6, h6]


def _expm1(x):
    """e^x - 1; NumPy's expm1 for real input, e^x - 1 for complex input (its
    imaginary part, which carries the complex-step derivative, suffers no
    cancellation)."""
    if np.iscomplexobj(x):
        return np.exp(x) - 1.0
    return np.expm1(x)


def _gate_step(prob: Problem, z):
    """One Rush-Larsen or implicit-Euler step (gated models only)."""
    if not gate_fields(prob):
        raise ValueError(f"{prob.scheme} needs a gated model (fk, bocf), got {prob.model}")
    dt = prob.dt
    k = rhs(prob, z)
    coef = gate_coefficients(prob, z)
    out = []
    for f, zf in enumerate(z):
        if f in coef:
            a, b = coef[f]
            if prob.scheme == "rush_larsen":
                x = a * dt
                out.append(zf * np.exp(x) + (b / a) * _expm1(x))
            else:
                out.append((zf + dt * b) / (1.0 - dt * a))
        else:
            out.append(zf + dt * k[f])
    return out


def _gate_pointwise(prob: Problem, z):
    """The pointwise part of one gate step: the non-gate fields' explicit
    Euler step on the reaction alone (the diffusion term is linear and is
    transposed separately) and each gate's Rush-Larsen or implicit-Euler
    update, exactly as `_gate_step` forms them."""
    dt = prob.dt
    n = reaction(prob, z)
    coef = gate_coefficients(prob, z)
    out = []
    for f, zf in enumerate(z):
        if f in coef:
            a, b = coef[f]
            if prob.scheme == "rush_larsen":
                x = a * dt
                out.append(zf * np.exp(x) + (b / a) * _expm1(x))
            else:
                out.append((zf + dt * b) / (1.0 - dt * a))
        else:
            out.append(zf + dt * n[f])
    return out


def _gate_step_adjoint(prob: Problem, z, lam, Lt):
    """lam_n for one gate step: the transposed pointwise Jacobian of
    `_gate_pointwise` (complex-step columns) applied to lam, plus
    dt L^T lam on the diffusive fields."""
    nv = len(z)
    base = [np.asarray(a, dtype=np.complex128) for a in z]
    out = []
    for l in range(nv):
        pert = list(base)
        pert[l] = base[l] + 1j * COMPLEX_STEP
        col = _gate_pointwise(prob, pert)
        acc = (np.imag(col[0]) / COMPLEX_STEP) * lam[0]
        for m in range(1, nv):
            acc = acc + (np.imag(col[m]) / COMPLEX_STEP) * lam[m]
        out.append(acc)
    for f, lt in Lt.items():
        out[f] = out[f] + (lt @ (prob.dt * lam[f]).ravel()).reshape(lam[f].shape)
    return out


def _one_step(prob: Problem, z):
    dt = prob.dt
    if prob.scheme in ("rush_larsen", "implicit_euler"):
        return _gate_step(prob, z)
    if prob.scheme == "euler":
        k1 = rhs(prob, z)
        return _axpy(z, dt, k1)
    if prob.scheme == "heun":
        h2 = dt * 0.5
        k1 = rhs(prob, z)
        k2 = rhs(prob, _axpy(z, dt, k1))
        return [zi + h2 * (a + b) for zi, a, b in zip(z, k1, k2)]
    h2 = dt * 0.5
    h6 = dt / 6.0
    k1 = rhs(prob, z)
    k2 = rhs(prob, _axpy(z, h2, k1))
    k3 = rhs(prob, _axpy(z, h2, k2))
    k4 = rhs(prob, _axpy(z, dt, k3))
    return [zi + h6 * (((a + 2.0 * b) + 2.0 * c) + d)
            for zi, a, b, c, d in zip(z, k1, k2, k3, k4)]


def _check_state(prob: Problem, z):
    nv = n_fields(prob.model)
    if len(z) != nv:
        raise ValueError(f"{prob.model} has {nv} fields, got {len(z)}")
    for a in z:
        if np.shape(a) != prob.shape:
            raise ValueError(f"field shape {np.shape(a)} != {prob.shape}")


def step(prob: Problem, z, nsteps: int = 1):
    """Advance state ``z`` (list of arrays of shape ``prob.shape``) by ``nsteps`` steps."""
    _check_state(prob, z)
    z = [np.array(a, copy=True) for a in z]
    for _ in range(int(nsteps)):
        z = _one_step(prob, z)
    return z


def stage_states(prob: Problem, z):
    """Stage inputs Y_1..Y_S of one step from state z."""
    A, _ = _coefficients(prob)
    ys, ks = [], []
    for s in range(len(A)):
        y = list(z)
        for j, a in enumerate(A[s]):
            if a != 0.0:
                y = _axpy(y, a, ks[j])
        ys.append(y)
        ks.append(rhs(prob, y))
    return ys


COMPLEX_STEP = 1e-30


def jvp(prob: Problem, z, dz, nsteps: int = 1):
    """(Phi(z), dPhi(z) . dz) over ``nsteps`` steps, by complex step."""
    _check_state(prob, z)
    _check_state(prob, dz)
    zc = [np.asarray(a, dtype=np.float64) + 1j * COMPLEX_STEP * np.asarray(b, dtype=np.float64)
          for a, b in zip(z, dz)]
    zc = step(prob, zc, nsteps)
    return step(prob, z, nsteps), [np.imag(c) / COMPLEX_STEP for c in zc]


def _jac_transpose(prob: Problem, Lt, y, a):
    nv = len(y)
    jac = reaction_jacobian(prob, y)
    out = []
    for l in range(nv):
        acc = jac[0][l] * a[0]
        for m in range(1, nv):
            acc = acc + jac[m][l] * a[m]
        out.append(acc)
    for f, lt in Lt.items():
        out[f] = out[f] + (lt @ a[f].ravel()).reshape(a[f].shape)
    return out


def step_adjoint(prob: Problem, z, lam, Lt=None):
    """lam_n = (dPhi/dz at z_n)^T lam_{n+1} for one step; Lt as returned by
    `transposed_operators`."""
    if Lt is None:
        Lt = transposed_operators(prob)
    if prob.scheme in ("rush_larsen", "implicit_euler"):
        return _gate_step_adjoint(prob, z, lam, Lt)
    A, B = _coefficients(prob)
    ys = stage_states(prob, z)
    S = len(B)
    zbar = [np.array(a, dtype=np.float64, copy=True) for a in lam]
    kbar = [[b * a for a in lam] for b in B]
    for s in reversed(range(S)):
        ybar = _jac_transpose(prob, Lt, ys[s], kbar[s])
        zbar = [zb + yb for zb, yb in zip(zbar, ybar)]
        for j, a in enumerate(A[s]):
            if a != 0.0:
                kbar[j] = [kb + a * yb for kb, yb in zip(kbar[j], ybar)]
    return zbar


def vjp(prob: Problem, z0, lam_T, nsteps: int, checkpoint_every: int = 64):
    """(dPhi^nsteps/dz at z0)^T lam_T, with states stored every
    ``checkpoint_every`` steps and recomputed within each segment."""
    _check_state(prob, z0)
    _check_state(prob, lam_T)
    nsteps = int(nsteps)
    C = int(checkpoint_every) if checkpoint_every and checkpoint_every > 0 else max(nsteps, 1)
    Lt = transposed_operators(prob)
    ckpts = []
    z = [np.array(a, dtype=np.float64, copy=True) for a in z0]
    for n in range(nsteps):
        if n % C == 0:
            ckpts.append(z)
        z = _one_step(prob, z)
    lam = [np.array(a, dtype=np.float64, copy=True) for a in lam_T]
    for seg in reversed(range(len(ckpts))):
        start = seg * C
        stop = min(start + C, nsteps)
        states = [ckpts[seg]]
        for _ in range(start, stop - 1):
            states.append(_one_step(prob, states[-1]))
        for n in reversed(range(start, stop)):
            lam = step_adjoint(prob, states[n - start], lam, Lt)
    return lam
