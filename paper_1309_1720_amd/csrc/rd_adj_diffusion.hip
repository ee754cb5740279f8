// Adjoint-step kernels of the diffusion model, 5- and 9-point stencils, all schemes.
#include "rd_adjoint.h"

namespace rd {
hipError_t launch_adjoint_diffusion(int stencil, int scheme, const AdjArgs& a, hipStream_t stream) {
  return launch_adjoint_model<RD_MODEL_DIFFUSION>(stencil, scheme, a, stream);
}
}  // namespace rd
