// rd_check.hip -- the optional finiteness check behind RD_ENONFINITE: after
// a call has enqueued its work, scan the fields it produced for NaN or
// infinity.  A debugging aid: the scan synchronises the caller's stream, so
// it is refused inside a stream capture.  Its one flag word lives in the last
// 256 bytes of the caller's workspace (the library allocates nothing).
#include <atomic>
#include <cstring>

#include "rd_host.h"

namespace rd {

static std::atomic<int> g_check_finite{0};

size_t check_finite_bytes() { return g_check_finite.load() ? 256 : 0; }

constexpr int kCheckArrays = 8;

struct FiniteArgs {
  const double* f[kCheckArrays];
  int nf;
  long long n;
  int* flag;
};

__global__ void finite_clear_kernel(int* flag) {
  if (threadIdx.x == 0) *flag = 0;
}

// Any lane that sees a non-finite value stores 1 (every writer stores the
// same value, so the races are benign).
__global__ __launch_bounds__(256) void finite_scan_kernel(FiniteArgs a) {
  bool bad = false;
  for (int f = 0; f < a.nf; ++f)
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < a.n; i += (long long)gridDim.x * 256)
      bad = bad || !__builtin_isfinite(a.f[f][i]);
  if (bad) *a.flag = 1;
}

int check_finite_allowed(hipStream_t s) {
  if (!g_check_finite.load()) return RD_OK;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  if (st != hipStreamCaptureStatusNone)
    return fail(RD_EUNSUPPORTED, "the finiteness check synchronises the stream; disable it during a capture");
  return RD_OK;
}

int check_finite(double* const* f, int nf, size_t n, char* flag_ws, hipStream_t s, const char* what) {
  if (!g_check_finite.load() || nf == 0 || n == 0) return RD_OK;
  int rc = check_finite_allowed(s);
  if (rc) return rc;
  int* flag = (int*)flag_ws;
  hipLaunchKernelGGL(finite_clear_kernel, dim3(1), dim3(64), 0, s, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "finite check launch");
  for (int f0 = 0; f0 < nf; f0 += kCheckArrays) {
    FiniteArgs a;
    std::memset(&a, 0, sizeof a);
    a.nf = nf - f0 < kCheckArrays ? nf - f0 : kCheckArrays;
    for (int k = 0; k < a.nf; ++k) a.f[k] = f[f0 + k];
    a.n = (long long)n;
    a.flag = flag;
    const long long blocks = ((long long)n + 255) / 256;
    hipLaunchKernelGGL(finite_scan_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "finite check launch");
  }
  int h = 0;
  e = hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "finite check copy");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "finite check synchronise");
  if (h) return fail(RD_ENONFINITE, "%s: the result holds NaN or infinite values", what);
  return RD_OK;
}

}  // namespace rd

extern "C" int rd_set_check_finite(int32_t enable) {
  rd::g_check_finite.store(enable != 0 ? 1 : 0);
  return RD_OK;
}
