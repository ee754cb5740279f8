// Fused reverse-step kernels (stage inputs recomputed in the adjoint sweep) of the fhn model.
#include "rd_adjoint_fused.h"

namespace rd {
hipError_t launch_adjoint_fused_fhn(int stencil, int scheme, const AdjFusedArgs& a, hipStream_t s) {
  return launch_adjoint_fused_model<RD_MODEL_FHN>(stencil, scheme, a, s);
}
}  // namespace rd
