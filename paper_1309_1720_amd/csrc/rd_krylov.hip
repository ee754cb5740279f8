// rd_krylov.hip -- vector algebra for matrix-free Krylov solvers built on
// rd_jvp / rd_step_batched (an addition to the paper, whose introduction
// motivates Newton-Krylov solves on the time-T flow, Sect. 1).
//
// A Krylov vector is one device array of n doubles (the fields of a state
// stored one after the other).  Two operations cover Arnoldi with classical
// Gram-Schmidt and the solution update:
//   gram:    out[k] = <x_k, w>,                     k < m
//   lincomb: y     = beta y + sum_k coef[k] x_k
// Both stream their operands once (HBM-bound) and sum in a fixed order, so
// results do not depend on timing.
#include <cstring>

#include "rd_host.h"

namespace rd {

constexpr int kKrylovMax = 64;     // vectors per call
constexpr int kGramChunk = 8;      // basis vectors per block pass (registers)
constexpr int kGramBlocks = 512;   // partial sums per vector
constexpr int kVecThreads = 256;

struct GramArgs {
  const double* x[kKrylovMax];
  const double* w;
  double* partial;  // [kGramBlocks][m]
  double* out;      // [m]
  long long n;
  int m;
};

// Block b accumulates, for a chunk of up to kGramChunk vectors (blockIdx.y),
// the products over its grid-stride share of the elements, then reduces
// them across the block in LDS in a fixed tree order.
__global__ __launch_bounds__(kVecThreads) void gram_partial_kernel(GramArgs a) {
  const int k0 = blockIdx.y * kGramChunk;
  const int nk = min(kGramChunk, a.m - k0);
  double acc[kGramChunk];
#pragma unroll
  for (int k = 0; k < kGramChunk; ++k) acc[k] = 0.0;
  for (long long i = (long long)blockIdx.x * kVecThreads + threadIdx.x; i < a.n;
       i += (long long)gridDim.x * kVecThreads) {
    const double wi = a.w[i];
#pragma unroll
    for (int k = 0; k < kGramChunk; ++k)
      if (k < nk) acc[k] = fma(a.x[k0 + k][i], wi, acc[k]);
  }
  __shared__ double red[kGramChunk][kVecThreads];
#pragma unroll
  for (int k = 0; k < kGramChunk; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = kVecThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < kGramChunk; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < nk) a.partial[(size_t)blockIdx.x * a.m + k0 + threadIdx.x] = red[threadIdx.x][0];
}

// Thread k sums the kGramBlocks partials of vector k in block order.
__global__ void gram_final_kernel(GramArgs a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.m) return;
  double s = 0.0;
  for (int b = 0; b < kGramBlocks; ++b) s += a.partial[(size_t)b * a.m + k];
  a.out[k] = s;
}

struct LincombArgs {
  const double* x[kKrylovMax];
  double coef[kKrylovMax];
  double* y;
  double beta;
  long long n;
  int m;
};

__global__ __launch_bounds__(kVecThreads) void lincomb_kernel(LincombArgs a) {
  for (long long i = (long long)blockIdx.x * kVecThreads + threadIdx.x; i < a.n;
       i += (long long)gridDim.x * kVecThreads) {
    double t = a.beta == 0.0 ? 0.0 : a.beta * a.y[i];
    for (int k = 0; k < a.m; ++k) t = fma(a.coef[k], a.x[k][i], t);
    a.y[i] = t;
  }
}

static int vec_blocks(long long n) {
  const long long b = (n + kVecThreads - 1) / kVecThreads;
  return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

}  // namespace rd

using namespace rd;

extern "C" {

int rd_vec_gram_workspace_bytes(int32_t m, size_t* out) {
  if (!out) return fail(RD_EINVAL, "out is NULL");
  if (m < 1 || m > kKrylovMax) return fail(RD_EINVAL, "m = %d outside [1, %d]", m, kKrylovMax);
  *out = (size_t)kGramBlocks * (size_t)m * sizeof(double);
  return RD_OK;
}

int rd_vec_gram(const double* const* x, int32_t m, const double* w, int64_t n, double* out, void* ws,
                size_t ws_bytes, void* hip_stream) {
  size_t need = 0;
  int rc = rd_vec_gram_workspace_bytes(m, &need);
  if (rc) return rc;
  if (!x || !w || !out) return fail(RD_EINVAL, "x, w and out must not be NULL");
  if (n < 1) return fail(RD_EINVAL, "n = %lld must be >= 1", (long long)n);
  if (!ws || ws_bytes < need)
    return fail(RD_EWORKSPACE, "workspace of %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, need);
  if (((uintptr_t)ws) % 8 != 0 || ((uintptr_t)w) % 8 != 0 || ((uintptr_t)out) % 8 != 0)
    return fail(RD_EINVAL, "pointers must be 8-byte aligned");
  GramArgs a;
  std::memset(&a, 0, sizeof a);
  for (int k = 0; k < m; ++k) {
    if (!x[k] || ((uintptr_t)x[k]) % 8 != 0) return fail(RD_EINVAL, "x[%d] is NULL or misaligned", k);
    a.x[k] = x[k];
  }
  a.w = w;
  a.partial = (double*)ws;
  a.out = out;
  a.n = n;
  a.m = m;
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(gram_partial_kernel, dim3(kGramBlocks, (m + kGramChunk - 1) / kGramChunk), dim3(kVecThreads),
                     0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "gram launch");
  hipLaunchKernelGGL(gram_final_kernel, dim3(1), dim3(kKrylovMax), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "gram reduction launch");
  return RD_OK;
}

int rd_vec_lincomb(double* y, double beta, const double* const* x, const double* coef, int32_t m, int64_t n,
                   void* hip_stream) {
  if (!y) return fail(RD_EINVAL, "y is NULL");
  if (m < 0 || m > kKrylovMax) return fail(RD_EINVAL, "m = %d outside [0, %d]", m, kKrylovMax);
  if (m > 0 && (!x || !coef)) return fail(RD_EINVAL, "x and coef must not be NULL");
  if (n < 1) return fail(RD_EINVAL, "n = %lld must be >= 1", (long long)n);
  if (((uintptr_t)y) % 8 != 0) return fail(RD_EINVAL, "y is not 8-byte aligned");
  LincombArgs a;
  std::memset(&a, 0, sizeof a);
  for (int k = 0; k < m; ++k) {
    if (!x[k] || ((uintptr_t)x[k]) % 8 != 0) return fail(RD_EINVAL, "x[%d] is NULL or misaligned", k);
    a.x[k] = x[k];
    a.coef[k] = coef[k];
  }
  a.y = y;
  a.beta = beta;
  a.n = n;
  a.m = m;
  hipLaunchKernelGGL(lincomb_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, (hipStream_t)hip_stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "lincomb launch");
  return RD_OK;
}

}  // extern "C"
