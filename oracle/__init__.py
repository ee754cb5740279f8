"""Plain, slow, CPU-only FP64 oracle for the explicit cardiac
reaction-diffusion step of Marcotte & Grigoriev, "Implementation of PDE
models of cardiac dynamics on GPUs using OpenCL" (arXiv:1309.1720).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the test suite, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP library
or its Python binding: it is NumPy written from the paper's equations.

Layout (whole-grid NumPy arrays of shape (ny, nx), or (nz, ny, nx) for the
3-D stencils, x fastest):
  * ``problem``   -- the oracle's own problem description.
  * ``stencils``  -- ghost cells (Fig. 1), the 5-point and isotropic
                     9-point Laplacians (Eq. 6), the anisotropic flux form,
                     the 3-D 7/19/27-point operators, and the same operators
                     assembled as sparse matrices.
  * ``models``    -- smoothed step H_k (Sect. 2) and the reaction terms
                     N[z] of Eq. (1): FitzHugh-Nagumo (Eq. 3, two diffusive
                     fields), Barkley, Fenton-Karma, Bueno-Orovio (Eq. 5),
                     and pure diffusion (N = 0).
  * ``integrate`` -- explicit Euler, Heun and classical RK4 (Sect. 3), the
                     Rush-Larsen and implicit-Euler gate steps (Sect. 3), the
                     tangent-linear map by complex-step differentiation of
                     the forward flow, and the adjoint by explicit
                     transposition of each stage.

Every function is dtype-generic (float64 or complex128) so that the
forward flow can be run in complex arithmetic; branches of the step
function are taken on the real part.
"""
from .problem import Problem
from .stencils import (ghost_pad, laplacian, lap5, lap9, lap3d, lap_aniso, fibre_coefficients,
                       laplacian_matrix, WEIGHTS_3D)
from .models import (smooth_step, reaction, reaction_jacobian, n_fields, diffusive_fields, gate_fields,
                     gate_coefficients)
from .integrate import rhs, step, jvp, vjp, step_adjoint, stage_states, transposed_operators

__all__ = [
    "Problem", "ghost_pad", "laplacian", "lap5", "lap9", "lap3d", "WEIGHTS_3D", "lap_aniso",
    "fibre_coefficients", "laplacian_matrix", "smooth_step", "reaction",
    "reaction_jacobian", "n_fields", "diffusive_fields", "gate_fields", "gate_coefficients", "rhs", "step", "jvp", "vjp",
    "step_adjoint", "stage_states", "transposed_operators",
]
