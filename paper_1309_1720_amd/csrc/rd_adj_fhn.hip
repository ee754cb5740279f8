// Adjoint-step kernels of the FitzHugh-Nagumo model, all stencils and schemes.
#include "rd_adjoint.h"

namespace rd {
hipError_t launch_adjoint_fhn(int stencil, int scheme, const AdjArgs& a, hipStream_t stream) {
  return launch_adjoint_model<RD_MODEL_FHN>(stencil, scheme, a, stream);
}
}  // namespace rd
