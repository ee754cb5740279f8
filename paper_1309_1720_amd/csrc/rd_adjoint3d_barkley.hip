// 3-D reverse-stage kernels, barkley model (rd_adjoint3d.h).
#include "rd_adjoint3d.h"

namespace rd {
hipError_t launch_adjoint3d_barkley(int stencil, int kind, const Adj3Args& a, hipStream_t s) {
  return launch_adjoint3d_model<RD_MODEL_BARKLEY>(stencil, kind, a, s);
}
}  // namespace rd
