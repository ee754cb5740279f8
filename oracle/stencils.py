"""Diffusion operators of the oracle (Marcotte & Grigoriev, Sect. 3).

Grid: cell-centred, x_i = (i + 1/2) dx, arrays indexed [j, i] (row j is y).

Boundary (Eq. 2, Fig. 1).  No-flux boundaries are imposed with one layer of
ghost cells that are assigned the value of the adjacent boundary cell, i.e.
the field is mirrored about the domain edge half a cell outside the last
cell centre.  Corner ghosts take the corner cell's value.

Isotropic 9-point Laplacian (Eq. 6).  The paper fixes the structure -- equal
axial weights alpha_a, equal diagonal weights alpha_d, and a balanced centre
alpha_00 = -4 (alpha_a + alpha_d) -- but prints no values.  Consistency with
the Laplacian requires alpha_a + 2 alpha_d = 1, and the rotational-symmetry
motive of Sect. 3 (an isotropic leading error term, (dx^2/12) lap^2 u) fixes
alpha_a = 4 alpha_d, hence alpha_a = 2/3 and alpha_d = 1/6.  The balanced
centre is applied by differencing each neighbour group against 4 U_ij, which
gives exactly zero on a uniform field.

5-point Laplacian: the canonical central-difference operator named in
Sect. 3, (W + E + N + S - 4 C) / dx^2.

Periodic boundaries (the alternative Sect. 3 describes: displacements that
leave the domain map to the opposite edge): ghost cells take the values of
the opposite edge, and in the flux form every face is interior, the face
between the last and the first column included (its tensor is that of
x = nx dx).

3-D stencils (the conclusion looks ahead to three-dimensional tissue; the
paper prints no 3-D operator).  Arrays are indexed [k, j, i] (k is z).  The
27 cells of the 3 x 3 x 3 block around a cell fall into faces (6, one
coordinate differs), edges (12, two differ) and corners (8, three differ);
L u = c (w_f (sum faces - 6 C) + w_e (sum edges - 12 C) + w_c (sum corners
- 8 C)), each group differenced against its own multiple of the centre as in
the 9-point operator.  Consistency requires w_f + 4 w_e + 4 w_c = 1 and an
isotropic leading error ((dx^2/12) lap^2 u, as for Eq. 6) requires
w_f = 2 w_e + 8 w_c: a one-parameter family in w_c, every member of which
reduces on a single plane with mirrored neighbours to the 2-D stencil of
Eq. 6 (axial 2/3, diagonal 1/6).
  lap7  : w = (1, 0, 0)            the canonical central difference
  lap19 : w = (1/3, 1/6, 0)        the isotropic member without corners
  lap27 : w = (7/15, 1/10, 1/30)   the compact (Mehrstellen) member
Ghost layers follow the 2-D rules in every direction (mirror for no-flux,
opposite face for periodic), corner and edge ghosts included.

Anisotropic tensor (extension of Eq. 1 to D = D_perp I + (D_par - D_perp) f f^T,
f = (cos theta, sin theta), theta linear in x).  Conservative flux form:
face fluxes F = D grad u on every interior face, zero flux on the domain
boundary faces (n . D grad u = 0), divergence of the face fluxes.  Cross
derivatives at a face use the four nearest cells across it, with the
ghost-cell mirror where a cross term reaches outside the domain.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .problem import Problem

ALPHA_AXIAL = 2.0 / 3.0
ALPHA_DIAG = 1.0 / 6.0
WEIGHTS_3D = {"lap7": (1.0, 0.0, 0.0), "lap19": (1.0 / 3.0, 1.0 / 6.0, 0.0),
              "lap27": (7.0 / 15.0, 1.0 / 10.0, 1.0 / 30.0)}


def ghost_pad(u: np.ndarray, bc: str = "noflux") -> np.ndarray:
    """Field with one ghost layer holding the adjacent boundary values (Fig. 1),
    or the opposite edge's values for periodic boundaries."""
    return np.pad(u, 1, mode="wrap" if bc == "periodic" else "edge")


def _neighbours(u, bc="noflux"):
    g = ghost_pad(u, bc)
    return {
        "C": g[1:-1, 1:-1], "W": g[1:-1, :-2], "E": g[1:-1, 2:],
        "N": g[:-2, 1:-1], "S": g[2:, 1:-1],
        "NW": g[:-2, :-2], "NE": g[:-2, 2:], "SW": g[2:, :-2], "SE": g[2:, 2:],
    }


def lap5(u: np.ndarray, c: float, bc: str = "noflux") -> np.ndarray:
    """c * (W + E + N + S - 4 C), c = D / dx^2."""
    n = _neighbours(u, bc)
    return c * (((n["W"] + n["E"]) + (n["N"] + n["S"])) - 4.0 * n["C"])


def lap9(u: np.ndarray, c: float, bc: str = "noflux") -> np.ndarray:
    """Balanced isotropic 9-point stencil of Eq. (6), c = D / (dx dy)."""
    n = _neighbours(u, bc)
    axial = ((n["W"] + n["E"]) + (n["N"] + n["S"])) - 4.0 * n["C"]
    diag = ((n["NW"] + n["SW"]) + (n["NE"] + n["SE"])) - 4.0 * n["C"]
    return c * (ALPHA_AXIAL * axial + ALPHA_DIAG * diag)


def fibre_coefficients(prob: Problem):
    """Tensor entries of D = D_perp I + (D_par - D_perp) f f^T.

    Returns (Dxx_f, Dxy_f, Dxy_c, Dyy_c): the first two at the interior
    x-faces i + 1/2 (i = 0 .. nx-2 of the window), the last two at the cell
    centres.  theta is linear in the global x coordinate, theta0 at x = 0
    and theta1 at x = nx_total dx.
    """
    n_tot = prob.n_total
    gi = np.arange(prob.nx, dtype=np.float64) + prob.x0
    dth = prob.theta1 - prob.theta0
    th_c = prob.theta0 + dth * ((gi + 0.5) / n_tot)
    th_f = prob.theta0 + dth * ((gi[:-1] + 1.0) / n_tot)
    dd = prob.D_par - prob.d_perp

    def tensor(th):
        c, s = np.cos(th), np.sin(th)
        return prob.d_perp + dd * c * c, dd * c * s, prob.d_perp + dd * s * s

    dxx_f, dxy_f, _ = tensor(th_f)
    _, dxy_c, dyy_c = tensor(th_c)
    return dxx_f, dxy_f, dxy_c, dyy_c


def lap_aniso(u: np.ndarray, prob: Problem, rel: float = 1.0) -> np.ndarray:
    """div(rel D grad u) in conservative flux form with zero boundary-face
    flux; the relative diffusivity rel scales the face-flux divergence."""
    if prob.bc == "periodic":
        return _lap_aniso_periodic(u, prob, rel)
    dxx_f, dxy_f, dxy_c, dyy_c = fibre_coefficients(prob)
    inv_dx2 = rel / (prob.dx * prob.dx)
    n = _neighbours(u)
    ny, nx = u.shape
    up, dn, we, ea = n["N"], n["S"], n["W"], n["E"]
    # x-faces between columns i and i+1: D_xx du/dx + D_xy du/dy (times dx).
    fx = (dxx_f * (u[:, 1:] - u[:, :-1])
          + (0.25 * dxy_f) * ((dn[:, 1:] + dn[:, :-1]) - (up[:, 1:] + up[:, :-1])))
    # y-faces between rows j and j+1: D_xy du/dx + D_yy du/dy (times dx).
    fy = ((0.25 * dxy_c) * ((ea[1:, :] + ea[:-1, :]) - (we[1:, :] + we[:-1, :]))
          + dyy_c * (u[1:, :] - u[:-1, :]))
    fx_all = np.zeros((ny, nx + 1), dtype=fx.dtype)
    fy_all = np.zeros((ny + 1, nx), dtype=fy.dtype)
    fx_all[:, 1:-1] = fx
    fy_all[1:-1, :] = fy
    return ((fx_all[:, 1:] - fx_all[:, :-1]) + (fy_all[1:, :] - fy_all[:-1, :])) * inv_dx2


def _periodic_tensor(prob: Problem):
    """(Dxx, Dxy) at the nx faces i + 1/2 (the last one at x = nx dx) and
    (Dxy, Dyy) at the centres, for the periodic flux form."""
    n_tot = prob.n_total
    gi = np.arange(prob.nx, dtype=np.float64) + prob.x0
    dth = prob.theta1 - prob.theta0
    th_c = prob.theta0 + dth * ((gi + 0.5) / n_tot)
    th_f = prob.theta0 + dth * ((gi + 1.0) / n_tot)
    dd = prob.D_par - prob.d_perp
    cf, sf, cc, sc = np.cos(th_f), np.sin(th_f), np.cos(th_c), np.sin(th_c)
    return prob.d_perp + dd * cf * cf, dd * cf * sf, dd * cc * sc, prob.d_perp + dd * sc * sc


def _lap_aniso_periodic(u: np.ndarray, prob: Problem, rel: float) -> np.ndarray:
    dxx_f, dxy_f, dxy_c, dyy_c = _periodic_tensor(prob)
    inv_dx2 = rel / (prob.dx * prob.dx)
    E = np.roll(u, -1, axis=1)            # u(i+1, j)
    W = np.roll(u, 1, axis=1)             # u(i-1, j)
    # x-face i+1/2 (between i and i+1, wrapping), all nx of them
    fx = (dxx_f * (E - u)
          + (0.25 * dxy_f) * ((np.roll(E, -1, axis=0) + np.roll(u, -1, axis=0))
                              - (np.roll(E, 1, axis=0) + np.roll(u, 1, axis=0))))
    # y-face j+1/2 (between j and j+1, wrapping), all ny of them
    fy = ((0.25 * dxy_c) * ((np.roll(E, -1, axis=0) + E) - (np.roll(W, -1, axis=0) + W))
          + dyy_c * (np.roll(u, -1, axis=0) - u))
    return ((fx - np.roll(fx, 1, axis=1)) + (fy - np.roll(fy, 1, axis=0))) * inv_dx2


def lap3d(u: np.ndarray, c: float, weights, bc: str = "noflux") -> np.ndarray:
    """3-D isotropic operator on an (nz, ny, nx) field:
    c (w_f (faces - 6 C) + w_e (edges - 12 C) + w_c (corners - 8 C)), groups
    with zero weight left out."""
    g = ghost_pad(u, bc)
    nz, ny, nx = u.shape
    centre = g[1:-1, 1:-1, 1:-1]
    sums = {1: 0.0, 2: 0.0, 3: 0.0}
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                m = abs(dk) + abs(dj) + abs(di)
                if m:
                    sums[m] = sums[m] + g[1 + dk:1 + dk + nz, 1 + dj:1 + dj + ny, 1 + di:1 + di + nx]
    count = {1: 6.0, 2: 12.0, 3: 8.0}
    out = 0.0
    for m, w in zip((1, 2, 3), weights):
        if w != 0.0:
            out = out + w * (sums[m] - count[m] * centre)
    return c * out


def laplacian(prob: Problem, u: np.ndarray, rel: float = 1.0) -> np.ndarray:
    """Diffusion term of a field with diffusivity rel * D_par (rel = 1: the
    voltage) for the problem's stencil and boundary condition."""
    if prob.is_3d:
        return lap3d(u, (prob.D_par * rel) / (prob.dx * prob.dx), WEIGHTS_3D[prob.stencil], prob.bc)
    if prob.stencil == "lap9_aniso":
        return lap_aniso(u, prob, rel)
    c = (prob.D_par * rel) / (prob.dx * prob.dx)
    if prob.stencil == "lap5":
        return lap5(u, c, prob.bc)
    return lap9(u, c, prob.bc)


# ---------------------------------------------------------------------------
# The same operators assembled as explicit sparse matrices (row-major flat
# index j * nx + i).  The adjoint uses their transposes.
# ---------------------------------------------------------------------------

def _clip(a, n):
    return np.clip(a, 0, n - 1)


def laplacian_matrix(prob: Problem, rel: float = 1.0) -> sp.csr_matrix:
    """The operator `laplacian(prob, ., rel)` as a sparse matrix."""
    if prob.bc == "periodic" or prob.is_3d:
        return _matrix_by_columns(prob, rel)
    nx, ny = prob.nx, prob.ny
    ncell = nx * ny
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    j, i = j.ravel(), i.ravel()
    me = j * nx + i
    rows, cols, vals = [], [], []

    def put(r, cidx, v):
        rows.append(np.asarray(r))
        cols.append(np.asarray(cidx))
        vals.append(np.broadcast_to(np.asarray(v, dtype=np.float64), np.shape(r)).copy())

    if prob.stencil in ("lap5", "lap9"):
        c = (prob.D_par * rel) / (prob.dx * prob.dx)
        axial = [(0, -1), (0, 1), (-1, 0), (1, 0)]
        diag = [(-1, -1), (1, -1), (-1, 1), (1, 1)]
        groups = [(axial, c * (1.0 if prob.stencil == "lap5" else ALPHA_AXIAL))]
        if prob.stencil == "lap9":
            groups.append((diag, c * ALPHA_DIAG))
        for offs, w in groups:
            for dj, di in offs:
                nb = _clip(j + dj, ny) * nx + _clip(i + di, nx)
                put(me, nb, w)
                put(me, me, -w)
        return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(ncell, ncell)).tocsr()

    # Anisotropic flux form: L = inv_dx2 * (Dx Gx + Dy Gy).
    dxx_f, dxy_f, dxy_c, dyy_c = fibre_coefficients(prob)
    inv_dx2 = rel / (prob.dx * prob.dx)
    # x-faces: index f = j * (nx - 1) + i for the face between i and i+1.
    nfx = ny * (nx - 1)
    fj, fi = np.meshgrid(np.arange(ny), np.arange(nx - 1), indexing="ij")
    fj, fi = fj.ravel(), fi.ravel()
    fidx = fj * (nx - 1) + fi
    gr, gc, gv = [], [], []

    def gput(r, cidx, v):
        gr.append(np.asarray(r))
        gc.append(np.asarray(cidx))
        gv.append(np.broadcast_to(np.asarray(v, dtype=np.float64), np.shape(r)).copy())

    if nfx:
        a = dxx_f[fi]
        q = 0.25 * dxy_f[fi]
        gput(fidx, fj * nx + fi + 1, a)
        gput(fidx, fj * nx + fi, -a)
        jp, jm = _clip(fj + 1, ny), _clip(fj - 1, ny)
        gput(fidx, jp * nx + fi + 1, q)
        gput(fidx, jp * nx + fi, q)
        gput(fidx, jm * nx + fi + 1, -q)
        gput(fidx, jm * nx + fi, -q)
        gx = sp.coo_matrix((np.concatenate(gv), (np.concatenate(gr), np.concatenate(gc))),
                           shape=(nfx, ncell)).tocsr()
        # divergence: cell (j,i) gets +F(i+1/2) - F(i-1/2)
        dr = np.concatenate([fj * nx + fi, fj * nx + fi + 1])
        dc = np.concatenate([fidx, fidx])
        dv = np.concatenate([np.ones(nfx), -np.ones(nfx)])
        dvx = sp.coo_matrix((dv, (dr, dc)), shape=(ncell, nfx)).tocsr()
        lx = dvx @ gx
    else:
        lx = sp.csr_matrix((ncell, ncell))

    nfy = (ny - 1) * nx
    gr, gc, gv = [], [], []
    if nfy:
        hj, hi = np.meshgrid(np.arange(ny - 1), np.arange(nx), indexing="ij")
        hj, hi = hj.ravel(), hi.ravel()
        hidx = hj * nx + hi
        b = dyy_c[hi]
        r = 0.25 * dxy_c[hi]
        gput(hidx, (hj + 1) * nx + hi, b)
        gput(hidx, hj * nx + hi, -b)
        ip, im = _clip(hi + 1, nx), _clip(hi - 1, nx)
        gput(hidx, (hj + 1) * nx + ip, r)
        gput(hidx, hj * nx + ip, r)
        gput(hidx, (hj + 1) * nx + im, -r)
        gput(hidx, hj * nx + im, -r)
        gy = sp.coo_matrix((np.concatenate(gv), (np.concatenate(gr), np.concatenate(gc))),
                           shape=(nfy, ncell)).tocsr()
        dr = np.concatenate([hj * nx + hi, (hj + 1) * nx + hi])
        dc = np.concatenate([hidx, hidx])
        dv = np.concatenate([np.ones(nfy), -np.ones(nfy)])
        dvy = sp.coo_matrix((dv, (dr, dc)), shape=(ncell, nfy)).tocsr()
        ly = dvy @ gy
    else:
        ly = sp.csr_matrix((ncell, ncell))
    return ((lx + ly) * inv_dx2).tocsr()


def _matrix_by_columns(prob: Problem, rel: float) -> sp.csr_matrix:
    """Periodic and 3-D operators, column by column: L e_k for every unit
    vector (small grids only; the adjoint tests use it)."""
    n = int(np.prod(prob.shape))
    cols = []
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        cols.append(sp.csr_matrix(laplacian(prob, e.reshape(prob.shape), rel).reshape(-1, 1)))
    return sp.hstack(cols).tocsr()
