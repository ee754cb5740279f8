// Fused-step kernels of the fk model advancing the state and a tangent, all stencils and schemes.
#include "rd_sweep.h"

namespace rd {
hipError_t launch_sweep_tan_fk(int stencil, int scheme, const SweepArgs& a, hipStream_t stream) {
  return launch_sweep_model<RD_MODEL_FENTON_KARMA, kModeTangent>(stencil, scheme, a, stream);
}
}  // namespace rd
