// Adjoint-step kernels of the fk model, all stencils and schemes.
#include "rd_adjoint.h"

namespace rd {
hipError_t launch_adjoint_fk(int stencil, int scheme, const AdjArgs& a, hipStream_t stream) {
  return launch_adjoint_model<RD_MODEL_FENTON_KARMA>(stencil, scheme, a, stream);
}
}  // namespace rd
