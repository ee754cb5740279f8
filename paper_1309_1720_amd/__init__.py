"""MI355X-native explicit time stepping of 2-D cardiac reaction-diffusion
models in FP64 (Marcotte & Grigoriev, arXiv:1309.1720).

The computation lives in the HIP library ``librd.so`` (C ABI in
``include/rd.h``); this package is its thin Python binding.  PyTorch provides
device memory and streams only.
"""
from ._binding import (  # noqa: F401
    ABI_VERSION, LIB_PATH, MODELS, N_FIELDS, SCHEMES, STENCILS, Problem, RDError,
    checkpoint_count, get_plan, get_steps_per_launch, get_tile_rows, jvp, lib, n_fields, n_params,
    release_workspaces, set_autotune, set_check_finite, set_fused_adjoint, set_kernel_variant, set_steps_per_launch, set_tile_rows, step,
    step_noalloc,
    step_batched, vec_gram, vec_lincomb, vjp, workspace_bytes,
)
from .autograd import RDFlow, flow  # noqa: F401,E402
from .krylov import gmres_lockstep, newton_krylov, periodic_orbit  # noqa: F401,E402
