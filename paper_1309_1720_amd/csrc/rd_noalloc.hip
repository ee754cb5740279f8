// rd_noalloc.hip -- rd_step_noalloc: rd_step whose scratch (the ping-pong
// partner of the state, and the finiteness-check flag) is a device array the
// library owns, for callers that cannot allocate device memory or pass a
// workspace.  Each GPU the library runs on holds its own copy of the array
// until the process ends.
#include <mutex>

#include "rd_host.h"

namespace rd {

constexpr size_t kNoallocScratchBytes = (size_t)RD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void* g_scratch[kMaxDevices];  // device address of `scratch`, per device

// The device the work of `stream` runs on (the current device for the null stream).
static int stream_device(hipStream_t stream, int* dev) {
  hipError_t e = stream ? hipStreamGetDevice(stream, dev) : hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, "looking up the stream's device");
  if (*dev < 0 || *dev >= kMaxDevices)
    return fail(RD_EUNSUPPORTED, "device %d is beyond the %d devices rd_step_noalloc tracks", *dev, kMaxDevices);
  return RD_OK;
}

// Address of device `dev`'s copy of `scratch`, looked up once per device with
// that device current (the host-side name `scratch` is not a device address).
static int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess && e2 != hipSuccess) return hip_fail(e2, "hipSetDevice");
    }
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(RD_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return RD_OK;
}

}  // namespace rd

using namespace rd;

extern "C" int rd_step_noalloc(const rd_problem* p, double* const* fields, double* checkpoints,
                               void* hip_stream) {
  int rc = validate(p);
  if (rc) return rc;
  size_t need = 0;
  rc = rd_workspace_bytes(p, RD_OP_STEP, &need);
  if (rc) return rc;
  if (need > kNoallocScratchBytes)
    return fail(RD_EWORKSPACE,
                "rd_step_noalloc: this problem needs %zu bytes of scratch, more than the %zu bytes the library "
                "holds per GPU; call rd_step with a workspace instead",
                need, kNoallocScratchBytes);
  int dev = -1;
  rc = stream_device((hipStream_t)hip_stream, &dev);
  if (rc) return rc;
  void* ws = nullptr;
  rc = scratch_address(dev, &ws);
  if (rc) return rc;
  return rd_step(p, fields, checkpoints, ws, kNoallocScratchBytes, hip_stream);
}
