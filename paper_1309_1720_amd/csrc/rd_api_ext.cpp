// Entry points still being brought up: they validate and report unsupported.
#include "rd_host.h"

namespace rd {
}  // namespace rd

using namespace rd;
extern "C" {
int rd_step_batched_workspace_bytes(const rd_problem*, int32_t, int32_t, size_t*) {
  return fail(RD_EUNSUPPORTED, "rd_step_batched is not available in this build");
}
int rd_step_batched(const rd_problem*, int32_t, double* const* const*, double* const* const*,
                    void*, size_t, void*) {
  return fail(RD_EUNSUPPORTED, "rd_step_batched is not available in this build");
}
}
