// Stage-pipelined fused-step kernels of the FitzHugh-Nagumo model advancing the state, all stencils and schemes.
#include "rd_pipe.h"

namespace rd {
hipError_t launch_pipe_fwd_fhn(int stencil, int scheme, const SweepArgs& a, hipStream_t stream) {
  return launch_pipe_model<RD_MODEL_FHN, kModeStep>(stencil, scheme, a, stream);
}
}  // namespace rd
