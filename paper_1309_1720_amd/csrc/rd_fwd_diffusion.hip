// Forward fused-step kernels of the diffusion model (all stencils and schemes).
#include "rd_fwd.h"

namespace rd {
hipError_t launch_fwd_diffusion(int stencil, int scheme, const FwdArgs& a, hipStream_t stream) {
  return launch_fwd_model<RD_MODEL_DIFFUSION>(stencil, scheme, a, stream);
}
}  // namespace rd
