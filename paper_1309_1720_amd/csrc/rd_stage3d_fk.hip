// 3-D stage kernels, fk model (rd_stage3d.h).
#include "rd_stage3d.h"

namespace rd {
hipError_t launch_stage3d_fk(int stencil, bool tangent, int kind, const Stage3Args& a, hipStream_t s) {
  return launch_stage3d_model<RD_MODEL_FENTON_KARMA>(stencil, tangent, kind, a, s);
}
}  // namespace rd
