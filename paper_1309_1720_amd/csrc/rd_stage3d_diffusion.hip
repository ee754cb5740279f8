// 3-D stage kernels, diffusion model (rd_stage3d.h).
#include "rd_stage3d.h"

namespace rd {
hipError_t launch_stage3d_diffusion(int stencil, bool tangent, int kind, const Stage3Args& a, hipStream_t s) {
  return launch_stage3d_model<RD_MODEL_DIFFUSION>(stencil, tangent, kind, a, s);
}
}  // namespace rd
