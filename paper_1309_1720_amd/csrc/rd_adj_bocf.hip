// Adjoint-step kernels of the bocf model, all stencils and schemes.
#include "rd_adjoint.h"

namespace rd {
hipError_t launch_adjoint_bocf(int stencil, int scheme, const AdjArgs& a, hipStream_t stream) {
  return launch_adjoint_model<RD_MODEL_BOCF>(stencil, scheme, a, stream);
}
}  // namespace rd
