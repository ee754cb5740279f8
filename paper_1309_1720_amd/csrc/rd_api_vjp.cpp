// rd_api_vjp.cpp -- rd_vjp: adjoint of the finite-time flow from stored
// checkpoints, recomputing the states of each checkpoint segment into the
// workspace and running the adjoint step kernel backwards through them.
#include <algorithm>
#include <cstring>

#include <atomic>

#include "rd_adjoint_fused.h"
#include "rd_host.h"

namespace rd {

hipError_t launch_adjoint_kernel(int model, int stencil, int scheme, const AdjArgs& a, hipStream_t s) {
  switch (model) {
    case RD_MODEL_DIFFUSION: return launch_adjoint_diffusion(stencil, scheme, a, s);
    case RD_MODEL_BARKLEY: return launch_adjoint_barkley(stencil, scheme, a, s);
    case RD_MODEL_FENTON_KARMA: return launch_adjoint_fk(stencil, scheme, a, s);
    case RD_MODEL_BOCF: return launch_adjoint_bocf(stencil, scheme, a, s);
    case RD_MODEL_FHN: return launch_adjoint_fhn(stencil, scheme, a, s);
  }
  return hipErrorInvalidValue;
}

static std::atomic<int> g_fused_adjoint{1};

static hipError_t launch_adjoint_fused_kernel(int model, int stencil, int scheme, const AdjFusedArgs& a,
                                              hipStream_t s) {
  switch (model) {
    case RD_MODEL_DIFFUSION: return launch_adjoint_fused_diffusion(stencil, scheme, a, s);
    case RD_MODEL_BARKLEY: return launch_adjoint_fused_barkley(stencil, scheme, a, s);
    case RD_MODEL_FHN: return launch_adjoint_fused_fhn(stencil, scheme, a, s);
  }
  return hipErrorInvalidValue;
}

// Whether rd_vjp's reverse step recomputes the stage inputs in the adjoint
// kernel (rd_adjoint_fused.h) for this problem.
bool fused_adjoint(const rd_problem* p) {
  return g_fused_adjoint.load() && n_fields(p->model) <= 2 && p->bc == RD_BC_NOFLUX && !is_3d(p->stencil) &&
         (p->scheme == RD_SCHEME_HEUN || p->scheme == RD_SCHEME_RK4);
}

// Workspace: (C - 1) recomputed states, NS - 1 stage inputs and one
// cotangent buffer, each n_fields arrays.
static size_t vjp_arrays(const rd_problem* p) {
  const size_t nv = (size_t)n_fields(p->model);
  const size_t C = (size_t)std::max(p->checkpoint_every, 1);
  return nv * ((C - 1) + (size_t)(n_stages(p->scheme) - 1) + 1);
}

int workspace_vjp(const rd_problem* p, size_t* out) {
  *out = is_3d(p->stencil) ? workspace_vjp_3d(p) : vjp_arrays(p) * field_bytes(p);
  return RD_OK;
}

}  // namespace rd

using namespace rd;

extern "C" int rd_set_fused_adjoint(int32_t enable) {
  g_fused_adjoint.store(enable != 0 ? 1 : 0);
  return RD_OK;
}

extern "C" int rd_vjp(const rd_problem* p, const double* checkpoints, double* const* cot, void* ws,
                      size_t ws_bytes, void* hip_stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = validate_fields(p, cot, "cotangents");
  if (rc) return rc;
  if (p->checkpoint_every <= 0) return fail(RD_EINVAL, "rd_vjp needs checkpoint_every > 0");
  if (p->nsteps == 0) return RD_OK;
  if (!checkpoints) return fail(RD_EINVAL, "checkpoints is NULL");
  if (((uintptr_t)checkpoints) % 8 != 0) return fail(RD_EINVAL, "checkpoints is not 8-byte aligned");
  size_t need = 0;
  workspace_vjp(p, &need);
  need += check_finite_bytes();
  char* flag = (char*)ws + (need - check_finite_bytes());
  if (!ws || ws_bytes < need)
    return fail(RD_EWORKSPACE, "workspace of %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, need);
  if (((uintptr_t)ws) % 256 != 0) return fail(RD_EINVAL, "workspace is not 256-byte aligned");
  rc = check_finite_allowed((hipStream_t)hip_stream);
  if (rc) return rc;

  if (is_3d(p->stencil)) {
    KConst c3;
    derive_constants(p, c3);
    rc = vjp_3d(p, c3, checkpoints, cot, (char*)ws, (hipStream_t)hip_stream);
    return rc ? rc
              : check_finite(cot, n_fields(p->model), (size_t)p->nx * p->ny * p->nz, flag, (hipStream_t)hip_stream,
                             "rd_vjp");
  }
  const int nv = n_fields(p->model);
  const int ns = n_stages(p->scheme);
  const int C = p->checkpoint_every;
  const size_t cells = (size_t)p->nx * (size_t)p->ny;
  const size_t fb = field_bytes(p);
  hipStream_t s = (hipStream_t)hip_stream;
  auto ws_array = [&](size_t i) { return (double*)((char*)ws + i * fb); };
  // layout: segment states [C-1][nv], stage inputs [ns-1][nv], cotangent buffer [nv]
  auto seg_state = [&](int i, int f) { return ws_array((size_t)i * nv + f); };
  auto stage_in = [&](int i, int f) { return ws_array((size_t)(C - 1) * nv + (size_t)i * nv + f); };
  double* lam_buf[kMaxFields];
  for (int f = 0; f < nv; ++f) lam_buf[f] = ws_array((size_t)(C - 1 + ns - 1) * nv + f);
  auto ckpt = [&](int64_t m, int f) { return (double*)checkpoints + ((size_t)m * nv + f) * cells; };

  KConst c;
  derive_constants(p, c);
  // recompute and stage-input launches use the forward step's plan; the
  // adjoint kernel its own band height
  const Plan fp = current_plan(kTuneForward, p->model, p->stencil, p->scheme, p->nx, p->ny, ns, true,
                               max_steps_per_launch(p->model, ns));
  KConst cf = c;
  cf.variant = fp.variant;
  cf.ksteps = 1;  // every intermediate state is needed
  set_geometry(cf, ns, fp.ty);
  // Adjoint band height: tuned on first use with trial launches that read the
  // caller's cotangent and first checkpoint and write only workspace (before
  // the workspace holds anything).
  auto adj_trial = [&](int ty) -> hipError_t {
    AdjArgs a;
    std::memset(&a, 0, sizeof a);
    a.c = c;
    set_geometry(a.c, ns, ty);
    for (int f = 0; f < nv; ++f) {
      a.z[f] = ckpt(0, f);
      a.lam_in[f] = cot[f];
      a.lam_out[f] = lam_buf[f];
    }
    for (int i = 0; i < ns - 1; ++i)
      for (int f = 0; f < nv; ++f) a.ys[i][f] = stage_in(i, f);
    return launch_adjoint_kernel(p->model, p->stencil, p->scheme, a, s);
  };
  const bool fused = fused_adjoint(p);
  KConst cfu = c;
  if (fused) {
    // the fused reverse step: its own band height, tuned the same way
    const int halo = fused_adjoint_halo(ns);
    auto fused_trial = [&](int ty) -> hipError_t {
      AdjFusedArgs a;
      std::memset(&a, 0, sizeof a);
      a.c = c;
      set_geometry(a.c, halo, ty);
      for (int f = 0; f < nv; ++f) {
        a.z[f] = ckpt(0, f);
        a.lam_in[f] = cot[f];
        a.lam_out[f] = lam_buf[f];
      }
      return launch_adjoint_fused_kernel(p->model, p->stencil, p->scheme, a, s);
    };
    set_geometry(cfu, halo,
                 tuned_rows(kTuneAdjointFused, p->model, p->stencil, p->scheme, p->nx, p->ny, halo, s, fused_trial));
  } else {
    set_geometry(c, ns, tuned_rows(kTuneAdjoint, p->model, p->stencil, p->scheme, p->nx, p->ny, ns, s, adj_trial));
  }

  double* curA[kMaxFields];
  double* curB[kMaxFields];
  for (int f = 0; f < nv; ++f) {
    curA[f] = cot[f];
    curB[f] = lam_buf[f];
  }
  double** cur = curA;
  double** oth = curB;
  if (p->nsteps % 2 == 1) {  // an odd number of swaps must end in the caller's arrays
    rc = copy_state(curB, curA, nv, cells * sizeof(double), s);
    if (rc) return rc;
    std::swap(cur, oth);
  }

  const int64_t nck = (p->nsteps + C - 1) / C;
  for (int64_t m = nck - 1; m >= 0; --m) {
    const int64_t start = m * C;
    const int64_t stop = std::min(start + (int64_t)C, p->nsteps);
    auto state = [&](int64_t n, int f) -> double* {
      return n == start ? ckpt(m, f) : seg_state((int)(n - start - 1), f);
    };
    // recompute z_{start+1} .. z_{stop-1}
    for (int64_t n = start + 1; n < stop; ++n) {
      SweepArgs a;
      std::memset(&a, 0, sizeof a);
      a.c = cf;
      for (int f = 0; f < nv; ++f) {
        a.in[f] = state(n - 1, f);
        a.out[f] = state(n, f);
      }
      hipError_t e = launch_sweep_mode(kModeStep, p->model, p->stencil, p->scheme, a, s);
      if (e != hipSuccess) return hip_fail(e, "recompute step launch");
    }
    for (int64_t n = stop - 1; n >= start; --n) {
      if (fused) {
        AdjFusedArgs a;
        std::memset(&a, 0, sizeof a);
        a.c = cfu;
        for (int f = 0; f < nv; ++f) {
          a.z[f] = state(n, f);
          a.lam_in[f] = cur[f];
          a.lam_out[f] = oth[f];
        }
        hipError_t e = launch_adjoint_fused_kernel(p->model, p->stencil, p->scheme, a, s);
        if (e != hipSuccess) return hip_fail(e, "fused adjoint step launch");
        std::swap(cur, oth);
        continue;
      }
      if (ns > 1) {
        SweepArgs a;
        std::memset(&a, 0, sizeof a);
        a.c = cf;
        for (int f = 0; f < nv; ++f) a.in[f] = state(n, f);
        for (int i = 0; i < ns - 1; ++i)
          for (int f = 0; f < nv; ++f) a.ys[i][f] = stage_in(i, f);
        hipError_t e = launch_sweep_mode(kModeStages, p->model, p->stencil, p->scheme, a, s);
        if (e != hipSuccess) return hip_fail(e, "stage-input launch");
      }
      AdjArgs a;
      std::memset(&a, 0, sizeof a);
      a.c = c;
      for (int f = 0; f < nv; ++f) {
        a.z[f] = state(n, f);
        a.lam_in[f] = cur[f];
        a.lam_out[f] = oth[f];
      }
      for (int i = 0; i < ns - 1; ++i)
        for (int f = 0; f < nv; ++f) a.ys[i][f] = stage_in(i, f);
      hipError_t e = launch_adjoint_kernel(p->model, p->stencil, p->scheme, a, s);
      if (e != hipSuccess) return hip_fail(e, "adjoint step launch");
      std::swap(cur, oth);
    }
  }
  return check_finite(cot, nv, cells, flag, s, "rd_vjp");
}
