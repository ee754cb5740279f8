// Adjoint-step kernels of the diffusion model, all stencils and schemes.
#include "rd_adjoint.h"

namespace rd {
hipError_t launch_adjoint_diffusion(int stencil, int scheme, const AdjArgs& a, hipStream_t stream) {
  return launch_adjoint_model<RD_MODEL_DIFFUSION>(stencil, scheme, a, stream);
}
}  // namespace rd
