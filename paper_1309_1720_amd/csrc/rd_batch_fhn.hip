// Batched fused-step kernels of the FitzHugh-Nagumo model (state, or state and tangent).
#include "rd_batch.h"

namespace rd {
hipError_t launch_batch_fhn(bool tangent, int stencil, int scheme, const BatchArgs& a, hipStream_t s) {
  return tangent ? launch_batch_model<RD_MODEL_FHN, kModeTangent>(stencil, scheme, a, s)
                 : launch_batch_model<RD_MODEL_FHN, kModeStep>(stencil, scheme, a, s);
}
}  // namespace rd
