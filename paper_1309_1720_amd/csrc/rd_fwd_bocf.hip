// Forward fused-step kernels of the bocf model (all stencils and schemes).
#include "rd_fwd.h"

namespace rd {
hipError_t launch_fwd_bocf(int stencil, int scheme, const FwdArgs& a, hipStream_t stream) {
  return launch_fwd_model<RD_MODEL_BOCF>(stencil, scheme, a, stream);
}
}  // namespace rd
