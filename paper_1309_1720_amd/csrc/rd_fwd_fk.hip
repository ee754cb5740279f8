// Forward fused-step kernels of the fk model (all stencils and schemes).
#include "rd_fwd.h"

namespace rd {
hipError_t launch_fwd_fk(int stencil, int scheme, const FwdArgs& a, hipStream_t stream) {
  return launch_fwd_model<RD_MODEL_FENTON_KARMA>(stencil, scheme, a, stream);
}
}  // namespace rd
