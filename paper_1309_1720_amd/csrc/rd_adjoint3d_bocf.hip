// 3-D reverse-stage kernels, bocf model (rd_adjoint3d.h).
#include "rd_adjoint3d.h"

namespace rd {
hipError_t launch_adjoint3d_bocf(int stencil, int kind, const Adj3Args& a, hipStream_t s) {
  return launch_adjoint3d_model<RD_MODEL_BOCF>(stencil, kind, a, s);
}
}  // namespace rd
