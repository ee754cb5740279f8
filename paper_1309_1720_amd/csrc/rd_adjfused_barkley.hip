// Fused reverse-step kernels (stage inputs recomputed in the adjoint sweep) of the barkley model.
#include "rd_adjoint_fused.h"

namespace rd {
hipError_t launch_adjoint_fused_barkley(int stencil, int scheme, const AdjFusedArgs& a, hipStream_t s) {
  return launch_adjoint_fused_model<RD_MODEL_BARKLEY>(stencil, scheme, a, s);
}
}  // namespace rd
