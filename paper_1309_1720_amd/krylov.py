"""Matrix-free Newton-Krylov solves on the time-T flow map (an addition to
the paper; its introduction motivates them: fixed points and periodic orbits
of the discretised flow are found by Newton's method whose linear systems
are solved by a Krylov method that needs only Jacobian-vector products).

For an ensemble of problems i (any sizes and models) the unknown is a state
z_i and the equation G_i(z_i) = Phi_i(z_i) - z_i = 0, with Phi_i the
nsteps-step flow of problem i.  Each Newton step solves (dPhi_i - I) dz_i =
-G_i with restarted GMRES; the GMRES iterations of all members advance in
lockstep, so each Krylov iteration is one batched launch sequence
(rd_step_batched with tangents) per group of members that share their
physics (everything but the grid size and the time step).  The
Jacobian-vector products are exact (tangent-linear kernels), or central
finite differences of two forward runs for comparison.  Vector algebra runs
in the library's kernels (rd_vec_gram, rd_vec_lincomb); the small Hessenberg
least-squares problems are solved on the host.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import _binding as B


def _views(flat: torch.Tensor, prob: B.Problem):
    return list(flat.view(prob.nfields, *prob.shape).unbind(0))


def _flat(fields) -> torch.Tensor:
    return torch.cat([f.reshape(-1) for f in fields])


def _physics(p: B.Problem):
    """What members of one rd_step_batched call must share (all but the grid
    size and the time step)."""
    return (p.model, p.scheme, p.stencil, p.dx, p.nsteps, p.D_par, p.D_perp, p.theta0, p.theta1,
            p.step_k, tuple(p.params), p.bc)


def _batched(probs, members, fields, tans=None) -> None:
    """rd_step_batched over `members`, one call per group of equal physics."""
    groups: dict = {}
    for k, i in enumerate(members):
        groups.setdefault(_physics(probs[i]), []).append(k)
    for ks in groups.values():
        B.step_batched([probs[members[k]] for k in ks], [fields[k] for k in ks],
                       None if tans is None else [tans[k] for k in ks])


def _norm(x: torch.Tensor) -> float:
    return float(B.vec_gram([x], x)[0].item()) ** 0.5


@dataclass
class GmresResult:
    x: list
    iterations: list
    residuals: list = field(default_factory=list)


def gmres_lockstep(matvec_many, bs, tol, restart: int = 30, max_cycles: int = 4) -> GmresResult:
    """Restarted GMRES for the systems A_i x_i = b_i, all advanced together.

    matvec_many(list of (i, v)) returns the list of A_i v.  tol[i] is the
    relative residual target of system i.  Arnoldi uses classical Gram-Schmidt
    applied twice (numerically as robust as modified Gram-Schmidt and two
    batched passes instead of j sequential ones)."""
    if not 1 <= restart <= 63:
        raise ValueError("restart must be in [1, 63] (at most 64 basis vectors per kernel call)")
    K = len(bs)
    xs = [torch.zeros_like(b) for b in bs]
    bnorm = [_norm(b) for b in bs]
    iters = [0] * K
    res = [1.0 if bn > 0 else 0.0 for bn in bnorm]
    for _cycle in range(max_cycles):
        active = [i for i in range(K) if bnorm[i] > 0 and res[i] > tol[i]]
        if not active:
            break
        # r = b - A x
        if any(iters[i] > 0 for i in active):
            ax = matvec_many([(i, xs[i]) for i in active])
            rs = {i: B.vec_lincomb(bs[i].clone(), 1.0, [a], [-1.0]) for i, a in zip(active, ax)}
        else:
            rs = {i: bs[i].clone() for i in active}
        beta = {i: _norm(rs[i]) for i in active}
        V = {i: [B.vec_lincomb(rs[i], 1.0 / beta[i])] for i in active}
        H = {i: np.zeros((restart + 1, restart)) for i in active}
        y = {}
        running = list(active)
        done_at = {}
        for j in range(restart):
            if not running:
                break
            ws = matvec_many([(i, V[i][j]) for i in running])
            still = []
            for i, w in zip(running, ws):
                h = B.vec_gram(V[i], w).cpu().numpy()
                B.vec_lincomb(w, 1.0, V[i], list(-h))
                h2 = B.vec_gram(V[i], w).cpu().numpy()
                B.vec_lincomb(w, 1.0, V[i], list(-h2))
                hn = _norm(w)
                H[i][: j + 1, j] = h + h2
                H[i][j + 1, j] = hn
                iters[i] += 1
                e1 = np.zeros(j + 2)
                e1[0] = beta[i]
                yi, *_ = np.linalg.lstsq(H[i][: j + 2, : j + 1], e1, rcond=None)
                rel = float(np.linalg.norm(e1 - H[i][: j + 2, : j + 1] @ yi)) / bnorm[i]
                y[i] = yi
                if rel <= tol[i] or hn == 0.0 or j == restart - 1:
                    done_at[i] = j + 1
                    res[i] = rel
                else:
                    V[i].append(B.vec_lincomb(w, 1.0 / hn))
                    still.append(i)
            running = still
        for i in active:
            m = done_at[i]
            B.vec_lincomb(xs[i], 1.0, V[i][:m], list(y[i]))
    return GmresResult(xs, iters, res)


@dataclass
class NewtonResult:
    states: list            # converged states (lists of field tensors)
    residuals: list         # per Newton iteration: max_i ||G_i|| / max(||z_i||, 1)
    krylov_iterations: list  # per Newton iteration: GMRES iterations per member


def newton_krylov(probs, states, tol: float = 1e-12, max_newton: int = 10, jvp: str = "exact",
                  fd_eps: float = 1e-7, restart: int = 30, max_cycles: int = 4) -> NewtonResult:
    """Fixed points of the nsteps-step flows: Phi_i(z_i) = z_i, from the
    starting states ``states`` (list per member of its field tensors).

    jvp = "exact": tangent-linear products (one batched state+tangent run);
    jvp = "fd":    (Phi(z + e v) - Phi(z - e v)) / (2 e), e = fd_eps * ||z|| / ||v||."""
    if jvp not in ("exact", "fd"):
        raise ValueError("jvp must be 'exact' or 'fd'")
    K = len(probs)
    z = [_flat(s).clone() for s in states]

    def flow(members, flats):
        """Phi applied to the given flat states (copies), batched."""
        fields = [_views(f.clone(), probs[i]) for i, f in zip(members, flats)]
        _batched(probs, members, fields)
        return [_flat(f) for f in fields]

    def matvec_many(pairs):
        members = [i for i, _ in pairs]
        if jvp == "exact":
            fields = [_views(z[i].clone(), probs[i]) for i in members]
            tans = [_views(v.clone(), probs[i]) for i, v in pairs]
            _batched(probs, members, fields, tans)
            outs = [_flat(t) for t in tans]
        else:
            eps = [fd_eps * max(_norm(z[i]), 1.0) / max(_norm(v), 1e-300) for i, v in pairs]
            plus = flow(members, [B.vec_lincomb(z[i].clone(), 1.0, [v], [e]) for (i, v), e in zip(pairs, eps)])
            minus = flow(members, [B.vec_lincomb(z[i].clone(), 1.0, [v], [-e]) for (i, v), e in zip(pairs, eps)])
            outs = [B.vec_lincomb(p, 0.5 / e, [m], [-0.5 / e]) for p, m, e in zip(plus, minus, eps)]
        return [B.vec_lincomb(o, 1.0, [v], [-1.0]) for o, (_, v) in zip(outs, pairs)]

    residuals, kits = [], []
    for _ in range(max_newton + 1):
        phi = flow(list(range(K)), z)
        g = [B.vec_lincomb(p, 1.0, [zi], [-1.0]) for p, zi in zip(phi, z)]
        rel = [_norm(gi) / max(_norm(zi), 1.0) for gi, zi in zip(g, z)]
        residuals.append(max(rel))
        if max(rel) <= tol or len(kits) == max_newton:
            break
        # inexact Newton: relative GMRES tolerance tied to the residual
        forcing = [min(1e-2, max(r, 1e-14) ** 0.5) for r in rel]
        rhs = [B.vec_lincomb(gi, -1.0) for gi in g]
        sol = gmres_lockstep(matvec_many, rhs, forcing, restart, max_cycles)
        kits.append(sol.iterations)
        for zi, dz in zip(z, sol.x):
            B.vec_lincomb(zi, 1.0, [dz], [1.0])
    return NewtonResult([_views(zi, p) for zi, p in zip(z, probs)], residuals, kits)


@dataclass
class PeriodicOrbitResult:
    states: list             # converged states (lists of field tensors)
    periods: list            # converged periods T_i
    residuals: list          # per Newton iteration: max_i ||Phi(z_i; T_i) - z_i|| / ||z_i||
    krylov_iterations: list  # per Newton iteration: GMRES iterations per member
    periods_history: list    # per Newton iteration: the periods it started from


def _with_period(prob: B.Problem, period: float) -> B.Problem:
    """The member's flow over time ``period``: its nsteps steps of dt = period / nsteps."""
    from dataclasses import replace
    return replace(prob, dt=float(period) / prob.nsteps, checkpoint_every=0)


def periodic_orbit(probs, states, periods, tol: float = 1e-10, max_newton: int = 16, jvp: str = "exact",
                   fd_eps: float = 1e-7, period_eps: float = 1e-6, restart: int = 60,
                   max_cycles: int = 4) -> PeriodicOrbitResult:
    """Periodic orbits of the discretised flow with unknown periods: states
    z_i and periods T_i with Phi(z_i; T_i) = z_i, where Phi(z; T) is member
    i's nsteps-step flow at the step dt = T / nsteps (nsteps fixed, so the
    period varies continuously).

    A periodic orbit is a one-parameter family (every point of the loop is a
    solution), so the flow direction is a null vector of dPhi - I.  Each
    Newton step solves the bordered system

        [ dPhi/dz - I   c ] [dz]   [-G]          G = Phi(z; T) - z,
        [ c^T           0 ] [dT] = [ 0],         c = dPhi/dT,

    whose last row is the phase condition: the correction is orthogonal to
    c, the flow direction at the orbit's end point (at convergence the flow
    direction at z itself), which removes the shift along the loop.  c is a
    central difference in T (two extra forward runs per Newton step); the
    products dPhi/dz v are the exact tangent-linear ones (jvp="exact": one
    batched state+tangent run per Krylov iteration, all members in lockstep)
    or central differences of two forward runs (jvp="fd", step fd_eps
    relative to ||z||), for comparison.  Bordered vectors are flat tensors
    of the member's state followed by one entry for T.
    """
    if jvp not in ("exact", "fd"):
        raise ValueError("jvp must be 'exact' or 'fd'")
    K = len(probs)
    if len(states) != K or len(periods) != K:
        raise ValueError("one state and one period per problem")
    z = [_flat(s).clone() for s in states]
    T = [float(t) for t in periods]
    n = [zi.numel() for zi in z]

    def flow(members, flats, period_of):
        fields = [_views(f.clone(), probs[i]) for i, f in zip(members, flats)]
        _batched([_with_period(probs[i], period_of(i)) for i in range(K)], members, fields)
        return [_flat(f) for f in fields]

    residuals, kits, thist = [], [], []
    for _ in range(max_newton + 1):
        members = list(range(K))
        phi = flow(members, z, lambda i: T[i])
        g = [B.vec_lincomb(p, 1.0, [zi], [-1.0]) for p, zi in zip(phi, z)]
        rel = [_norm(gi) / max(_norm(zi), 1.0) for gi, zi in zip(g, z)]
        residuals.append(max(rel))
        thist.append(list(T))
        if max(rel) <= tol or len(kits) == max_newton:
            break
        # c = dPhi/dT by a central difference in T
        hp = [T[i] * (1.0 + period_eps) for i in members]
        hm = [T[i] * (1.0 - period_eps) for i in members]
        plus = flow(members, z, lambda i: hp[i])
        minus = flow(members, z, lambda i: hm[i])
        cvec = [B.vec_lincomb(p, 1.0 / (hp[i] - hm[i]), [m], [-1.0 / (hp[i] - hm[i])])
                for i, (p, m) in enumerate(zip(plus, minus))]
        zprobs = [_with_period(probs[i], T[i]) for i in members]

        def matvec_many(pairs):
            idx = [i for i, _ in pairs]
            vz = [v[: n[i]] for i, v in pairs]
            if jvp == "exact":
                fields = [_views(z[i].clone(), probs[i]) for i in idx]
                tans = [_views(v.clone(), probs[i]) for i, v in zip(idx, vz)]
                _batched(zprobs, idx, fields, tans)
                jv = [_flat(t) for t in tans]
            else:
                eps = [fd_eps * max(_norm(z[i]), 1.0) / max(_norm(v), 1e-300) for i, v in zip(idx, vz)]
                fp = flow(idx, [B.vec_lincomb(z[i].clone(), 1.0, [v], [e]) for i, v, e in zip(idx, vz, eps)],
                          lambda i: T[i])
                fm = flow(idx, [B.vec_lincomb(z[i].clone(), 1.0, [v], [-e]) for i, v, e in zip(idx, vz, eps)],
                          lambda i: T[i])
                jv = [B.vec_lincomb(p, 0.5 / e, [m], [-0.5 / e]) for p, m, e in zip(fp, fm, eps)]
            out = []
            for (m, v), j, vzi in zip(pairs, jv, vz):
                vt = float(v[n[m]].item())
                B.vec_lincomb(j, 1.0, [vzi, cvec[m]], [-1.0, vt])   # (dPhi - I) vz + c vT
                out.append(torch.cat([j, B.vec_gram([cvec[m]], vzi)]))  # phase row <c, vz>
            return out

        forcing = [min(1e-2, max(r, 1e-14) ** 0.5) for r in rel]
        rhs = [torch.cat([B.vec_lincomb(gi.clone(), -1.0), torch.zeros(1, dtype=gi.dtype, device=gi.device)])
               for gi in g]
        sol = gmres_lockstep(matvec_many, rhs, forcing, restart, max_cycles)
        kits.append(sol.iterations)
        for i, dx in enumerate(sol.x):
            B.vec_lincomb(z[i], 1.0, [dx[: n[i]].contiguous()], [1.0])
            T[i] += float(dx[n[i]].item())
    return PeriodicOrbitResult([_views(zi, p) for zi, p in zip(z, probs)], T, residuals, kits, thist)
