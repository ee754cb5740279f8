// rd_api.cpp -- host runtime behind the C ABI of include/rd.h: argument
// validation, derived constants, launch geometry, workspace layout and the
// step loops that enqueue the fused kernels on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "rd_sweep.h"
#include "rd_host.h"

namespace rd {

static thread_local std::string g_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(RD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int n_fields(int model) {
  switch (model) {
    case RD_MODEL_DIFFUSION: return 1;
    case RD_MODEL_BARKLEY: return 2;
    case RD_MODEL_FENTON_KARMA: return 3;
    case RD_MODEL_BOCF: return 4;
    case RD_MODEL_FHN: return 2;
  }
  return RD_EINVAL;
}

int n_params(int model) {
  switch (model) {
    case RD_MODEL_DIFFUSION: return 0;
    case RD_MODEL_BARKLEY: return 3;
    case RD_MODEL_FENTON_KARMA: return 13;
    case RD_MODEL_BOCF: return 28;
    case RD_MODEL_FHN: return 4;
  }
  return RD_EINVAL;
}

int n_stages(int scheme) {
  switch (scheme) {
    case RD_SCHEME_EULER: return 1;
    case RD_SCHEME_HEUN: return 2;
    case RD_SCHEME_RK4: return 4;
    case RD_SCHEME_RUSH_LARSEN:
    case RD_SCHEME_IMPLICIT_EULER: return 1;
  }
  return RD_EINVAL;
}

bool gate_scheme(int scheme) { return scheme == RD_SCHEME_RUSH_LARSEN || scheme == RD_SCHEME_IMPLICIT_EULER; }

static bool finite(double x) { return std::isfinite(x); }

int validate(const rd_problem* p) {
  if (!p) return fail(RD_EINVAL, "problem is NULL");
  if (p->abi_version != RD_ABI_VERSION)
    return fail(RD_EINVAL, "abi_version %u, library has %d", p->abi_version, RD_ABI_VERSION);
  if (n_fields(p->model) < 0) return fail(RD_EINVAL, "unknown model %d", p->model);
  if (n_stages(p->scheme) < 0) return fail(RD_EINVAL, "unknown scheme %d", p->scheme);
  if (gate_scheme(p->scheme) && p->model != RD_MODEL_FENTON_KARMA && p->model != RD_MODEL_BOCF)
    return fail(RD_EUNSUPPORTED, "the Rush-Larsen and implicit-Euler schemes need a gated model (Fenton-Karma, Bueno-Orovio)");
  if (p->stencil != RD_LAP5 && p->stencil != RD_LAP9 && p->stencil != RD_LAP9_ANISO && !is_3d(p->stencil))
    return fail(RD_EINVAL, "unknown stencil %d", p->stencil);
  if (p->bc != RD_BC_NOFLUX && p->bc != RD_BC_PERIODIC) return fail(RD_EINVAL, "unknown boundary condition %d", p->bc);
  if (p->nx < 1 || p->ny < 1) return fail(RD_EINVAL, "grid %d x %d: both sides must be >= 1", p->nx, p->ny);
  if ((int64_t)p->nx * (int64_t)p->ny >= ((int64_t)1 << 31))
    return fail(RD_EINVAL, "grid %d x %d has 2^31 cells or more", p->nx, p->ny);
  if (is_3d(p->stencil)) {
    if (p->nz < 1) return fail(RD_EINVAL, "nz = %d must be >= 1", p->nz);
    if ((int64_t)p->nx * (int64_t)p->ny * (int64_t)p->nz >= ((int64_t)1 << 40))
      return fail(RD_EINVAL, "grid %d x %d x %d has 2^40 cells or more", p->nx, p->ny, p->nz);
  } else if (p->nz != 1) {
    return fail(RD_EINVAL, "nz = %d: the 2-D stencils need nz = 1", p->nz);
  }
  if (!(finite(p->dx) && p->dx > 0.0)) return fail(RD_EINVAL, "dx must be finite and > 0");
  if (!(finite(p->dt) && p->dt > 0.0)) return fail(RD_EINVAL, "dt must be finite and > 0");
  if (p->nsteps < 0) return fail(RD_EINVAL, "nsteps must be >= 0");
  if (!(finite(p->D_par) && p->D_par >= 0.0)) return fail(RD_EINVAL, "D_par must be finite and >= 0");
  if (p->stencil == RD_LAP9_ANISO) {
    if (!(finite(p->D_perp) && p->D_perp >= 0.0))
      return fail(RD_EINVAL, "D_perp must be finite and >= 0");
    if (!finite(p->theta0) || !finite(p->theta1)) return fail(RD_EINVAL, "fibre angles must be finite");
  }
  if (!(p->step_k > 0.0)) return fail(RD_EINVAL, "step_k must be > 0 (or +inf)");
  if (p->nparams != n_params(p->model))
    return fail(RD_EINVAL, "model %d takes %d parameters, got %d", p->model, n_params(p->model), p->nparams);
  if (p->nparams > 0 && !p->params) return fail(RD_EINVAL, "params is NULL");
  for (int i = 0; i < p->nparams; ++i)
    if (!finite(p->params[i])) return fail(RD_EINVAL, "parameter %d is not finite", i);
  if (p->model == RD_MODEL_FHN && p->params[0] < 0.0)
    return fail(RD_EINVAL, "FitzHugh-Nagumo delta (relative diffusivity of v) must be >= 0");
  if (p->checkpoint_every < 0) return fail(RD_EINVAL, "checkpoint_every must be >= 0");
  return RD_OK;
}

int validate_fields(const rd_problem* p, double* const* f, const char* what) {
  if (!f) return fail(RD_EINVAL, "%s array is NULL", what);
  const int nv = n_fields(p->model);
  for (int i = 0; i < nv; ++i) {
    if (!f[i]) return fail(RD_EINVAL, "%s[%d] is NULL", what, i);
    if (((uintptr_t)f[i]) % 8 != 0) return fail(RD_EINVAL, "%s[%d] is not 8-byte aligned", what, i);
  }
  for (int i = 0; i < nv; ++i)
    for (int j = i + 1; j < nv; ++j)
      if (f[i] == f[j]) return fail(RD_EINVAL, "%s[%d] and %s[%d] alias", what, i, what, j);
  return RD_OK;
}

// Model constants exactly as the equations are written: constant divisors
// become reciprocals, differences of constants are formed once.
void derive_constants(const rd_problem* p, KConst& c) {
  std::memset(&c, 0, sizeof c);
  c.nx = p->nx;
  c.ny = p->ny;
  c.ksteps = 1;
  c.periodic = p->bc == RD_BC_PERIODIC ? 1 : 0;
  c.sharp = std::isinf(p->step_k) ? 1 : 0;
  c.k = p->step_k;
  c.k6 = c.sharp ? 0.0 : 6.0 * p->step_k;
  c.dt = p->dt;
  c.h2 = p->dt * 0.5;
  c.h6 = p->dt / 6.0;
  // relative diffusivities of the diffusive fields: u 1, FitzHugh-Nagumo's v delta
  const double rel[2] = {1.0, p->model == RD_MODEL_FHN ? p->params[0] : 0.0};
  for (int d = 0; d < 2; ++d)
    c.dcoef[d] = p->stencil == RD_LAP9_ANISO ? rel[d] / (p->dx * p->dx) : (p->D_par * rel[d]) / (p->dx * p->dx);
  c.theta0 = p->theta0;
  c.dtheta = p->theta1 - p->theta0;
  c.n_total = (double)p->nx;
  c.d_perp = p->stencil == RD_LAP9_ANISO ? p->D_perp : p->D_par;
  c.dd = p->D_par - c.d_perp;
  const double* q = p->params;
  switch (p->model) {
    case RD_MODEL_FHN: {
      FhnC& m = c.m.fh;  // q = (delta, eps, a1, a0); delta scales dcoef[1]
      m.eps = q[1];
      m.a1 = q[2];
      m.a0 = q[3];
      break;
    }
    case RD_MODEL_BARKLEY: {
      BarkleyC& m = c.m.bk;
      m.b = q[1];
      m.inv_a = 1.0 / q[0];
      m.inv_eps = 1.0 / q[2];
      break;
    }
    case RD_MODEL_FENTON_KARMA: {
      // tau_v+, tau_v1-, tau_v2-, tau_w+, tau_w-, tau_d, tau_0, tau_r, tau_si, k_si, u_csi, u_c, u_v
      FentonKarmaC& m = c.m.fk;
      m.inv_tau_vp = 1.0 / q[0];
      m.tau_v2m = q[2];
      m.dtau_vm = q[1] - q[2];
      m.inv_tau_wp = 1.0 / q[3];
      m.inv_tau_wm = 1.0 / q[4];
      m.inv_tau_d = 1.0 / q[5];
      m.inv_tau_0 = 1.0 / q[6];
      m.inv_tau_r = 1.0 / q[7];
      m.inv_tau_si = 1.0 / q[8];
      m.lg_a = -2.0 * q[9];
      m.lg_b = 2.0 * q[9] * q[10];
      m.u_c = q[11];
      m.u_v = q[12];
      break;
    }
    case RD_MODEL_BOCF: {
      BocfC& m = c.m.bo;
      m.u_o = q[0];
      m.u_u = q[1];
      m.th_v = q[2];
      m.th_w = q[3];
      m.th_vm = q[4];
      m.th_o = q[5];
      m.tau_v1m = q[6];
      m.dtau_vm = q[7] - q[6];
      m.inv_tau_vp = 1.0 / q[8];
      m.tau_w1m = q[9];
      m.tau_w2m = q[10];
      m.lg_wm_a = -2.0 * q[11];
      m.lg_wm_b = 2.0 * q[11] * q[12];
      m.inv_tau_wp = 1.0 / q[13];
      m.inv_tau_fi = 1.0 / q[14];
      m.tau_o1 = q[15];
      m.dtau_o = q[16] - q[15];
      m.tau_so1 = q[17];
      m.tau_so2 = q[18];
      m.lg_so_a = -2.0 * q[19];
      m.lg_so_b = 2.0 * q[19] * q[20];
      m.tau_s1 = q[21];
      m.dtau_s = q[22] - q[21];
      m.lg_s_a = -2.0 * q[23];
      m.lg_s_b = 2.0 * q[23] * q[24];
      m.inv_tau_si = 1.0 / q[25];
      m.inv_tau_winf = 1.0 / q[26];
      m.w_infstar = q[27];
      break;
    }
    default:
      break;
  }
}

// Launch geometry for `ty` rows per wave band: column strips of 64 - 2 ns
// outputs, bands of ty rows.
void set_geometry(KConst& c, int halo, int ty) {
  const int tx = strip_width(halo);
  c.nsx = (c.nx + tx - 1) / tx;
  ty = std::max(1, std::min(ty, c.ny));
  c.ty = ty;
  c.nby = (c.ny + ty - 1) / ty;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t field_bytes(const rd_problem* p) {
  const size_t nz = is_3d(p->stencil) ? (size_t)p->nz : 1;
  return align_up((size_t)p->nx * (size_t)p->ny * nz * sizeof(double), 256);
}

hipError_t launch_sweep_mode(int mode, int model, int stencil, int scheme, const SweepArgs& a,
                             hipStream_t s) {
#define RD_MODE_SWITCH(name)                                                                       \
  switch (mode) {                                                                                  \
    case kModeStep:                                                                                \
      return pipe ? launch_pipe_fwd_##name(stencil, scheme, a, s) : launch_sweep_fwd_##name(stencil, scheme, a, s); \
    case kModeTangent:                                                                             \
      return pipe ? launch_pipe_tan_##name(stencil, scheme, a, s) : launch_sweep_tan_##name(stencil, scheme, a, s); \
    case kModeStages:                                                                              \
      return pipe ? launch_pipe_stg_##name(stencil, scheme, a, s) : launch_sweep_stg_##name(stencil, scheme, a, s); \
  }                                                                                                \
  break;
  // the pipelined variant handles neither the gate schemes nor periodic rows
  const bool pipe = a.c.variant == kVariantPipe && !gate_scheme(scheme) && !a.c.periodic;
  switch (model) {
    case RD_MODEL_DIFFUSION: RD_MODE_SWITCH(diffusion)
    case RD_MODEL_BARKLEY: RD_MODE_SWITCH(barkley)
    case RD_MODEL_FENTON_KARMA: RD_MODE_SWITCH(fk)
    case RD_MODEL_BOCF: RD_MODE_SWITCH(bocf)
    case RD_MODEL_FHN: RD_MODE_SWITCH(fhn)
  }
#undef RD_MODE_SWITCH
  return hipErrorInvalidValue;
}

int copy_state(double* const* dst, double* const* src, int nv, size_t bytes, hipStream_t s) {
  for (int f = 0; f < nv; ++f) {
    hipError_t e = hipMemcpyAsync(dst[f], src[f], bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  return RD_OK;
}

int max_steps_per_launch(int model, int ns) {
  return (model == RD_MODEL_DIFFUSION || model == RD_MODEL_BARKLEY || model == RD_MODEL_FHN) ? 8 / ns : 1;
}
static_assert(MultiStep<RD_MODEL_BARKLEY, 1, kModeStep>::max == 8 &&
                  MultiStep<RD_MODEL_DIFFUSION, 2, kModeStep>::max == 4 &&
                  MultiStep<RD_MODEL_BARKLEY, 4, kModeStep>::max == 2 &&
                  MultiStep<RD_MODEL_FHN, 2, kModeStep>::max == 4 &&
                  MultiStep<RD_MODEL_FENTON_KARMA, 1, kModeStep>::max == 1 &&
                  MultiStep<RD_MODEL_BARKLEY, 4, kModeTangent>::max == 1,
              "max_steps_per_launch must agree with MultiStep");

// nsteps fused steps of the packed arrays `a` (np = NV state fields, or 2 NV
// with the tangent fields after them), in place, ping-ponging through the
// equally sized buffers `b`; optional state checkpoints every `every` steps.
// Launches advance c.ksteps steps where that neither passes nsteps nor a
// checkpoint, and one step otherwise.
int run_steps(const rd_problem* p, const KConst& c, bool tangent, double* const* a,
              double* const* b, int64_t nsteps, double* checkpoints, int every, hipStream_t s) {
  const int nv = n_fields(p->model);
  const int np = tangent ? 2 * nv : nv;
  const size_t cells = (size_t)p->nx * (size_t)p->ny;
  const size_t bytes = cells * sizeof(double);
  const int K = tangent ? 1 : std::max(c.ksteps, 1);
  KConst c1 = c;  // one step per launch
  c1.ksteps = 1;
  set_geometry(c1, n_stages(p->scheme), c.ty);
  const bool ck = checkpoints && every > 0;
  auto chunk = [&](int64_t n) -> int {
    if (K > 1 && n + K <= nsteps && (!ck || n % every + K <= every)) return K;
    return 1;
  };
  int64_t launches = 0;
  for (int64_t n = 0; n < nsteps; n += chunk(n)) ++launches;

  double* bufA[kMaxPacked];
  double* bufB[kMaxPacked];
  for (int f = 0; f < np; ++f) {
    bufA[f] = a[f];
    bufB[f] = b[f];
  }
  double** cur = bufA;
  double** oth = bufB;
  if (launches % 2 == 1) {  // an odd number of launches must end in the caller's arrays
    int rc = copy_state(bufB, bufA, np, bytes, s);
    if (rc) return rc;
    cur = bufB;
    oth = bufA;
  }
  SweepArgs args;
  std::memset(&args, 0, sizeof args);
  for (int64_t n = 0; n < nsteps;) {
    if (ck && n % every == 0) {
      double* dst[kMaxFields];
      for (int f = 0; f < nv; ++f) dst[f] = checkpoints + ((size_t)(n / every) * nv + f) * cells;
      int rc = copy_state(dst, cur, nv, bytes, s);
      if (rc) return rc;
    }
    const int kk = chunk(n);
    args.c = kk == K ? c : c1;
    for (int f = 0; f < np; ++f) {
      args.in[f] = cur[f];
      args.out[f] = oth[f];
    }
    hipError_t e = launch_sweep_mode(tangent ? kModeTangent : kModeStep, p->model, p->stencil, p->scheme, args, s);
    if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    std::swap(cur, oth);
    n += kk;
  }
  return RD_OK;
}

// Chooses the band height for (problem, mode) -- tuning on first use with
// trial launches from `in` into `out` -- and stores the geometry in `c`.
void plan_geometry(const rd_problem* p, KConst& c, bool tangent, double* const* in,
                   double* const* out, hipStream_t s) {
  const int ns = n_stages(p->scheme);
  const int np = (tangent ? 2 : 1) * n_fields(p->model);
  const int kmax = tangent ? 1 : max_steps_per_launch(p->model, ns);
  auto trial = [&](Plan pl) {
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.c = c;
    a.c.variant = pl.variant;
    a.c.ksteps = pl.k;
    set_geometry(a.c, ns * pl.k, pl.ty);
    for (int f = 0; f < np; ++f) {
      a.in[f] = in[f];
      a.out[f] = out[f];
    }
    return launch_sweep_mode(tangent ? kModeTangent : kModeStep, p->model, p->stencil, p->scheme, a, s);
  };
  const Plan pl = tuned_plan(tangent ? kTuneTangent : kTuneForward, p->model, p->stencil, p->scheme,
                             p->nx, p->ny, ns, s, trial, !gate_scheme(p->scheme) && p->bc == RD_BC_NOFLUX,
                             0, 0, kmax);
  c.variant = pl.variant;
  c.ksteps = pl.k;
  set_geometry(c, ns * pl.k, pl.ty);
}

int check_workspace(void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return RD_OK;
  if (!ws || ws_bytes < need)
    return fail(RD_EWORKSPACE, "workspace of %zu bytes, need %zu", ws ? ws_bytes : (size_t)0, need);
  if (((uintptr_t)ws) % 256 != 0) return fail(RD_EINVAL, "workspace is not 256-byte aligned");
  return RD_OK;
}

int workspace_jvp(const rd_problem* p, size_t* out) {
  *out = 2 * (size_t)n_fields(p->model) * field_bytes(p);
  return RD_OK;
}

}  // namespace rd

using namespace rd;

extern "C" {

int rd_abi_version(void) { return RD_ABI_VERSION; }

int rd_n_fields(int32_t model) {
  int n = n_fields(model);
  if (n < 0) return fail(RD_EINVAL, "unknown model %d", model);
  return n;
}

int rd_n_params(int32_t model) {
  int n = n_params(model);
  if (n < 0) return fail(RD_EINVAL, "unknown model %d", model);
  return n;
}

const char* rd_last_error(void) { return g_error.c_str(); }

int rd_checkpoint_count(const rd_problem* p, int64_t* out) {
  int rc = validate(p);
  if (rc) return rc;
  if (!out) return fail(RD_EINVAL, "out is NULL");
  *out = p->checkpoint_every > 0 ? (p->nsteps + p->checkpoint_every - 1) / p->checkpoint_every : 0;
  return RD_OK;
}

int rd_workspace_bytes(const rd_problem* p, int32_t op, size_t* out) {
  if (op == RD_OP_BATCHED || op == RD_OP_BATCHED_JVP) {
    // the batch p[0 .. nbatch-1], nbatch read from *out
    if (!out) return fail(RD_EINVAL, "out is NULL");
    const size_t n = *out;
    if (n < 1 || n > 65536)
      return fail(RD_EINVAL, "batched workspace query: *out must hold nbatch in [1, 65536] on entry, got %zu", n);
    return batch_workspace(p, (int32_t)n, op == RD_OP_BATCHED_JVP, out);
  }
  int rc = validate(p);
  if (rc) return rc;
  if (!out) return fail(RD_EINVAL, "out is NULL");
  const size_t nv = (size_t)n_fields(p->model);
  const size_t fb = field_bytes(p);
  if (is_3d(p->stencil)) {
    switch (op) {
      case RD_OP_STEP: *out = workspace_3d(p, false) + check_finite_bytes(); return RD_OK;
      case RD_OP_JVP: *out = workspace_3d(p, true) + check_finite_bytes(); return RD_OK;
      case RD_OP_VJP: *out = workspace_vjp_3d(p) + check_finite_bytes(); return RD_OK;
    }
    return fail(RD_EINVAL, "unknown op %d", op);
  }
  switch (op) {
    case RD_OP_STEP: *out = nv * fb + check_finite_bytes(); return RD_OK;
    case RD_OP_JVP:
      workspace_jvp(p, out);
      *out += check_finite_bytes();
      return RD_OK;
    case RD_OP_VJP:
      workspace_vjp(p, out);
      *out += check_finite_bytes();
      return RD_OK;
  }
  return fail(RD_EINVAL, "unknown op %d", op);
}

int rd_step(const rd_problem* p, double* const* fields, double* checkpoints, void* ws,
            size_t ws_bytes, void* hip_stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = validate_fields(p, fields, "fields");
  if (rc) return rc;
  if (checkpoints && ((uintptr_t)checkpoints) % 8 != 0)
    return fail(RD_EINVAL, "checkpoints is not 8-byte aligned");
  if (p->nsteps == 0) return RD_OK;
  size_t need = 0;
  rd_workspace_bytes(p, RD_OP_STEP, &need);
  rc = check_workspace(ws, ws_bytes, need);
  if (rc) return rc;
  rc = check_finite_allowed((hipStream_t)hip_stream);
  if (rc) return rc;
  const int nv = n_fields(p->model);
  hipStream_t s = (hipStream_t)hip_stream;
  KConst c;
  derive_constants(p, c);
  char* flag = (char*)ws + (need - check_finite_bytes());
  const size_t cells = (size_t)p->nx * (size_t)p->ny * (size_t)(is_3d(p->stencil) ? p->nz : 1);
  if (is_3d(p->stencil)) {
    rc = run_steps_3d(p, c, false, fields, (char*)ws, p->nsteps, checkpoints, p->checkpoint_every, s);
    return rc ? rc : check_finite(fields, nv, cells, flag, s, "rd_step");
  }
  double* b[kMaxFields];
  for (int f = 0; f < nv; ++f) b[f] = (double*)((char*)ws + f * field_bytes(p));
  plan_geometry(p, c, false, fields, b, s);
  rc = run_steps(p, c, false, fields, b, p->nsteps, checkpoints, p->checkpoint_every, s);
  return rc ? rc : check_finite(fields, nv, cells, flag, s, "rd_step");
}

int rd_jvp(const rd_problem* p, double* const* fields, double* const* tangents, void* ws,
           size_t ws_bytes, void* hip_stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = validate_fields(p, fields, "fields");
  if (rc) return rc;
  rc = validate_fields(p, tangents, "tangents");
  if (rc) return rc;
  const int nv = n_fields(p->model);
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j)
      if (fields[i] == tangents[j]) return fail(RD_EINVAL, "fields[%d] aliases tangents[%d]", i, j);
  if (p->nsteps == 0) return RD_OK;
  size_t need = 0;
  rd_workspace_bytes(p, RD_OP_JVP, &need);
  rc = check_workspace(ws, ws_bytes, need);
  if (rc) return rc;
  rc = check_finite_allowed((hipStream_t)hip_stream);
  if (rc) return rc;
  double* a[kMaxPacked];
  double* b[kMaxPacked];
  for (int f = 0; f < nv; ++f) {
    a[f] = fields[f];
    a[nv + f] = tangents[f];
  }
  for (int f = 0; f < 2 * nv; ++f) b[f] = (double*)((char*)ws + f * field_bytes(p));
  hipStream_t s = (hipStream_t)hip_stream;
  KConst c;
  derive_constants(p, c);
  char* flag = (char*)ws + (need - check_finite_bytes());
  const size_t cells = (size_t)p->nx * (size_t)p->ny * (size_t)(is_3d(p->stencil) ? p->nz : 1);
  if (is_3d(p->stencil)) {
    rc = run_steps_3d(p, c, true, a, (char*)ws, p->nsteps, nullptr, 0, s);
  } else {
    plan_geometry(p, c, true, a, b, s);
    rc = run_steps(p, c, true, a, b, p->nsteps, nullptr, 0, s);
  }
  return rc ? rc : check_finite(a, 2 * nv, cells, flag, s, "rd_jvp");
}

}  // extern "C"
