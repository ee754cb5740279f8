// 3-D reverse-stage kernels, diffusion model (rd_adjoint3d.h).
#include "rd_adjoint3d.h"

namespace rd {
hipError_t launch_adjoint3d_diffusion(int stencil, int kind, const Adj3Args& a, hipStream_t s) {
  return launch_adjoint3d_model<RD_MODEL_DIFFUSION>(stencil, kind, a, s);
}
}  // namespace rd
