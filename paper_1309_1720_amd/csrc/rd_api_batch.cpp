// rd_api_batch.cpp -- rd_step_batched: validation, workspace layout and the
// launch sequence (descriptor setup, optional copy, one launch per step).
#include <algorithm>
#include <cstring>
#include <vector>

#include "rd_batch.h"
#include "rd_host.h"

namespace rd {

static hipError_t launch_batch_kernel(bool tangent, int model, int stencil, int scheme,
                                      const BatchArgs& a, hipStream_t s) {
  switch (model) {
    case RD_MODEL_DIFFUSION: return launch_batch_diffusion(tangent, stencil, scheme, a, s);
    case RD_MODEL_BARKLEY: return launch_batch_barkley(tangent, stencil, scheme, a, s);
    case RD_MODEL_FENTON_KARMA: return launch_batch_fk(tangent, stencil, scheme, a, s);
    case RD_MODEL_BOCF: return launch_batch_bocf(tangent, stencil, scheme, a, s);
    case RD_MODEL_FHN: return launch_batch_fhn(tangent, stencil, scheme, a, s);
  }
  return hipErrorInvalidValue;
}

// Everything except the grid size and the time step must agree across the batch.
static int check_uniform(const rd_problem* probs, int32_t n) {
  const rd_problem& q = probs[0];
  for (int32_t i = 1; i < n; ++i) {
    const rd_problem& p = probs[i];
    const bool aniso = q.stencil == RD_LAP9_ANISO;
    if (p.model != q.model || p.scheme != q.scheme || p.stencil != q.stencil || p.bc != q.bc ||
        p.dx != q.dx || p.nsteps != q.nsteps || p.D_par != q.D_par ||
        p.step_k != q.step_k || p.nparams != q.nparams ||
        (aniso && (p.D_perp != q.D_perp || p.theta0 != q.theta0 || p.theta1 != q.theta1)))
      return fail(RD_EUNSUPPORTED, "problem %d differs from problem 0 in more than its grid size and time step", i);
    if (q.nparams > 0 && std::memcmp(p.params, q.params, sizeof(double) * q.nparams) != 0)
      return fail(RD_EUNSUPPORTED, "problem %d has different model parameters from problem 0", i);
  }
  return RD_OK;
}

static size_t table_bytes(int32_t n) { return align_up(sizeof(BatchInst) * (size_t)n, 256); }

// 2-D: the descriptor table and one partner array per instance array.  3-D:
// each instance's own stage workspace (its grids run one after another).
int batch_workspace(const rd_problem* probs, int32_t n, bool tangent, size_t* out) {
  if (!probs) return fail(RD_EINVAL, "problems is NULL");
  if (n < 1 || n > 65536) return fail(RD_EINVAL, "nbatch %d outside [1, 65536]", n);
  size_t total = is_3d(probs[0].stencil) ? 0 : table_bytes(n);
  for (int32_t i = 0; i < n; ++i) {
    int rc = validate(&probs[i]);
    if (rc) return fail(rc, "problem %d: %s", i, rd_last_error());
    if (is_3d(probs[i].stencil))
      total += workspace_3d(&probs[i], tangent);
    else
      total += (tangent ? 2 : 1) * (size_t)n_fields(probs[i].model) * field_bytes(&probs[i]);
  }
  *out = total + check_finite_bytes();
  return RD_OK;
}

}  // namespace rd

using namespace rd;

extern "C" int rd_step_batched_workspace_bytes(const rd_problem* probs, int32_t nbatch,
                                               int32_t with_tangents, size_t* out) {
  if (!out) return fail(RD_EINVAL, "out is NULL");
  size_t n = nbatch > 0 ? (size_t)nbatch : 0;
  const int rc = rd_workspace_bytes(probs, with_tangents ? RD_OP_BATCHED_JVP : RD_OP_BATCHED, &n);
  if (rc == RD_OK) *out = n;
  return rc;
}

// The 2-D batch: one descriptor table and one launch per step over all
// instances (see the kernel in rd_batch.h).
static int run_batched_2d(const rd_problem* probs, int32_t nbatch, double* const* const* fields,
                          double* const* const* tangents, void* ws, hipStream_t s) {
  const bool tangent = tangents != nullptr;
  const rd_problem& q = probs[0];
  const int nv = n_fields(q.model);
  const int nf = (tangent ? 2 : 1) * nv;
  const int ns = n_stages(q.scheme);
  BatchInst* table = (BatchInst*)ws;
  std::vector<BatchInst> inst(nbatch);
  char* next = (char*)ws + table_bytes(nbatch);
  int max_nx = 1, max_ny = 1;
  uint32_t shape_hash = 2166136261u;
  for (int32_t i = 0; i < nbatch; ++i) {
    BatchInst& I = inst[i];
    std::memset(&I, 0, sizeof I);
    I.nx = probs[i].nx;
    I.ny = probs[i].ny;
    // the time-step constants exactly as derive_constants forms them
    KConst ci;
    derive_constants(&probs[i], ci);
    I.dt = ci.dt;
    I.h2 = ci.h2;
    I.h6 = ci.h6;
    for (int f = 0; f < nf; ++f) {
      I.a[f] = f < nv ? fields[i][f] : tangents[i][f - nv];
      I.b[f] = (double*)next;
      next += field_bytes(&probs[i]);
    }
    max_nx = std::max(max_nx, I.nx);
    max_ny = std::max(max_ny, I.ny);
    shape_hash = (shape_hash ^ (uint32_t)I.nx) * 16777619u;
    shape_hash = (shape_hash ^ (uint32_t)I.ny) * 16777619u;
  }

  BatchArgs args;
  std::memset(&args, 0, sizeof args);
  derive_constants(&q, args.c);
  args.table = table;
  args.ninst = nbatch;
  args.nf = nf;

  // Per-instance geometry for `ty` rows per band, and the table upload.
  auto plan = [&](int ty) -> hipError_t {
    int waves = 0;
    for (auto& I : inst) {
      KConst g;
      g.nx = I.nx;
      g.ny = I.ny;
      set_geometry(g, ns, ty);
      I.nsx = g.nsx;
      I.nby = g.nby;
      I.ty = g.ty;
      I.wave_begin = waves;
      waves += g.nsx * g.nby;
    }
    args.total_waves = waves;
    for (int32_t first = 0; first < nbatch; first += kInstPerSetup) {
      BatchSetupArgs sa;
      std::memset(&sa, 0, sizeof sa);
      sa.table = table;
      sa.first = first;
      sa.count = std::min(kInstPerSetup, nbatch - first);
      for (int k = 0; k < sa.count; ++k) sa.inst[k] = inst[first + k];
      hipLaunchKernelGGL(batch_setup_kernel, dim3(1), dim3(kInstPerSetup), 0, s, sa);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  auto trial = [&](int ty) -> hipError_t {
    hipError_t e = plan(ty);
    if (e != hipSuccess) return e;
    args.parity = 0;  // reads the caller's arrays, writes workspace only
    return launch_batch_kernel(tangent, q.model, q.stencil, q.scheme, args, s);
  };
  // Untuned start: the tallest bands that still give every SIMD a few waves.
  auto total_waves = [&](int ty) {
    long long w = 0;
    for (auto& I : inst) {
      KConst g;
      g.nx = I.nx;
      g.ny = I.ny;
      set_geometry(g, ns, ty);
      w += (long long)g.nsx * g.nby;
    }
    return w;
  };
  int start_ty = 4;
  for (int ty : {64, 48, 32, 24, 16, 12, 8, 6})
    if (total_waves(ty) >= 4096) {
      start_ty = ty;
      break;
    }
  const int ty = tuned_rows(kTuneBatched + (tangent ? 8 : 0), q.model, q.stencil, q.scheme, max_nx, max_ny,
                            ns, s, trial, (int)(shape_hash & 0x7fffffff), start_ty);
  hipError_t e = plan(ty);
  if (e != hipSuccess) return hip_fail(e, "batch table setup");

  int parity = 0;
  if (q.nsteps % 2 == 1) {  // an odd number of steps must end in the caller's arrays
    BatchCopyArgs ca{table, nf};
    hipLaunchKernelGGL(batch_copy_kernel, dim3(64, nbatch), dim3(256), 0, s, ca);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batch copy launch");
    parity = 1;
  }
  for (int64_t n = 0; n < q.nsteps; ++n) {
    args.parity = parity;
    e = launch_batch_kernel(tangent, q.model, q.stencil, q.scheme, args, s);
    if (e != hipSuccess) return hip_fail(e, "batched step launch");
    parity ^= 1;
  }
  return RD_OK;
}

extern "C" int rd_step_batched(const rd_problem* probs, int32_t nbatch, double* const* const* fields,
                               double* const* const* tangents, void* ws, size_t ws_bytes,
                               void* hip_stream) {
  const bool tangent = tangents != nullptr;
  size_t need = 0;
  int rc = batch_workspace(probs, nbatch, tangent, &need);
  if (rc) return rc;
  rc = check_uniform(probs, nbatch);
  if (rc) return rc;
  if (!fields) return fail(RD_EINVAL, "fields is NULL");
  const rd_problem& q = probs[0];
  const int nv = n_fields(q.model);
  const int nf = (tangent ? 2 : 1) * nv;
  for (int32_t i = 0; i < nbatch; ++i) {
    rc = validate_fields(&probs[i], fields[i], "fields");
    if (rc) return fail(rc, "problem %d: %s", i, rd_last_error());
    if (tangent) {
      rc = validate_fields(&probs[i], tangents[i], "tangents");
      if (rc) return fail(rc, "problem %d: %s", i, rd_last_error());
    }
  }
  if (q.nsteps == 0) return RD_OK;
  if (!ws || ws_bytes < need)
    return fail(RD_EWORKSPACE, "workspace of %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, need);
  if (((uintptr_t)ws) % 256 != 0) return fail(RD_EINVAL, "workspace is not 256-byte aligned");
  rc = check_finite_allowed((hipStream_t)hip_stream);
  if (rc) return rc;

  hipStream_t s = (hipStream_t)hip_stream;
  if (is_3d(q.stencil)) {
    // 3-D grids: each instance's stage launches in turn (every instance is
    // large enough to fill the GPU on its own), bit-identical to rd_step and
    // rd_jvp on it
    char* w = (char*)ws;
    for (int32_t i = 0; i < nbatch; ++i) {
      KConst ci;
      derive_constants(&probs[i], ci);
      double* a[2 * kMaxFields];
      for (int f = 0; f < nf; ++f) a[f] = f < nv ? fields[i][f] : tangents[i][f - nv];
      rc = run_steps_3d(&probs[i], ci, tangent, a, w, q.nsteps, nullptr, 0, s);
      if (rc) return fail(rc, "problem %d: %s", i, rd_last_error());
      w += workspace_3d(&probs[i], tangent);
    }
  } else {
    rc = run_batched_2d(probs, nbatch, fields, tangents, ws, s);
    if (rc) return rc;
  }
  if (check_finite_bytes()) {
    char* flag = (char*)ws + (need - check_finite_bytes());
    for (int32_t i = 0; i < nbatch; ++i) {
      const size_t cells = (size_t)probs[i].nx * (size_t)probs[i].ny * (size_t)(is_3d(q.stencil) ? probs[i].nz : 1);
      double* arrs[2 * kMaxFields];
      for (int f = 0; f < nv; ++f) {
        arrs[f] = fields[i][f];
        if (tangent) arrs[nv + f] = tangents[i][f];
      }
      int rc2 = check_finite(arrs, tangent ? 2 * nv : nv, cells, flag, s, "rd_step_batched");
      if (rc2) return fail(rc2, "problem %d: %s", i, rd_last_error());
    }
  }
  return RD_OK;
}
