"""The oracle's own description of one integration problem.

Mirrors the problem statement of Sect. 3: a model, its parameters, an
N x N (here nx x ny) Cartesian grid of spacing dx = dy, a fixed time step
dt and no-flux boundaries (Eq. 2).  The 3-D stencils (lap7, lap19, lap27)
take an nx x ny x nz grid of the same spacing in all three directions;
their states are arrays of shape (nz, ny, nx).  ``x0``/``nx_total`` place a cropped
window inside a larger domain (used only to evaluate the fibre angle of the
anisotropic tensor at global coordinates).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MODELS = ("diffusion", "barkley", "fk", "bocf", "fhn")
SCHEMES = ("euler", "heun", "rk4", "rush_larsen", "implicit_euler")
STENCILS = ("lap5", "lap9", "lap9_aniso", "lap7", "lap19", "lap27")
STENCILS_3D = ("lap7", "lap19", "lap27")
BCS = ("noflux", "periodic")


@dataclass(frozen=True)
class Problem:
    model: str
    scheme: str
    stencil: str
    nx: int
    ny: int
    dx: float
    dt: float
    D_par: float = 1.0
    D_perp: float | None = None
    theta0: float = 0.0
    theta1: float = 0.0
    step_k: float = 28.4
    params: tuple = field(default_factory=tuple)
    x0: int = 0
    nx_total: int | None = None
    bc: str = "noflux"
    nz: int = 1

    def __post_init__(self):
        if self.model not in MODELS:
            raise ValueError(f"unknown model {self.model!r}")
        if self.scheme not in SCHEMES:
            raise ValueError(f"unknown scheme {self.scheme!r}")
        if self.stencil not in STENCILS:
            raise ValueError(f"unknown stencil {self.stencil!r}")
        if self.bc not in BCS:
            raise ValueError(f"unknown boundary condition {self.bc!r}")
        if self.nz != 1 and self.stencil not in STENCILS_3D:
            raise ValueError(f"nz = {self.nz} needs a 3-D stencil, got {self.stencil!r}")
        object.__setattr__(self, "params", tuple(float(p) for p in self.params))

    @property
    def d_perp(self) -> float:
        return self.D_par if self.D_perp is None else self.D_perp

    @property
    def is_3d(self) -> bool:
        return self.stencil in STENCILS_3D

    @property
    def shape(self) -> tuple:
        """Shape of one field: (nz, ny, nx) for the 3-D stencils, else (ny, nx)."""
        return (self.nz, self.ny, self.nx) if self.is_3d else (self.ny, self.nx)

    @property
    def n_total(self) -> int:
        return self.nx if self.nx_total is None else self.nx_total

    @classmethod
    def from_workload(cls, w: dict, params=None, **overrides) -> "Problem":
        keys = ("model", "scheme", "stencil", "nx", "ny", "dx", "dt", "D_par",
                "D_perp", "theta0", "theta1", "step_k", "bc", "nz")
        kw = {k: w[k] for k in keys if k in w}
        kw["params"] = tuple(np.asarray(params, dtype=np.float64)) if params is not None else ()
        kw.update(overrides)
        return cls(**kw)
