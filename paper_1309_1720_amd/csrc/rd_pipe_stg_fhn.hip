// Stage-pipelined fused-step kernels of the FitzHugh-Nagumo model producing the stage inputs of a step, all stencils and schemes.
#include "rd_pipe.h"

namespace rd {
hipError_t launch_pipe_stg_fhn(int stencil, int scheme, const SweepArgs& a, hipStream_t stream) {
  return launch_pipe_model<RD_MODEL_FHN, kModeStages>(stencil, scheme, a, stream);
}
}  // namespace rd
