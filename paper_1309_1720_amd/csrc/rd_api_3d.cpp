// rd_api_3d.cpp -- host side of the 3-D stencils: launch geometry, workspace
// layout, the stage sequence of each scheme (rd_stage3d.h) and the adjoint's
// reverse stages (rd_adjoint3d.h).
#include <algorithm>
#include <cstring>

#include "rd_adjoint3d.h"
#include "rd_host.h"
#include "rd_stage3d.h"

namespace rd {

bool is_3d(int stencil) { return stencil == RD_LAP7 || stencil == RD_LAP19 || stencil == RD_LAP27; }

// Workgroup grid: 64-column strips x groups of four rows x chunks of zc
// planes, with enough chunks for about 8192 wavefronts (32 per CU) and at
// least four planes per chunk (each chunk reads two extra planes).
template <class Args>
static void geometry_3d(const rd_problem* p, Args& a) {
  a.nz = p->nz;
  a.nbx = (p->nx + kStage3Width - 1) / kStage3Width;
  a.nby = (p->ny + kStage3Waves - 1) / kStage3Waves;
  const long long layer = (long long)a.nbx * p->ny;  // wavefronts per chunk layer
  long long nbz = (8192 + layer - 1) / layer;
  nbz = std::max(1LL, std::min(nbz, (long long)(p->nz + 3) / 4));
  a.zc = (int)((p->nz + nbz - 1) / nbz);
  a.nbz = (p->nz + a.zc - 1) / a.zc;
}

static hipError_t launch_stage(int model, int stencil, bool tangent, int kind, const Stage3Args& a,
                               hipStream_t s) {
  switch (model) {
    case RD_MODEL_DIFFUSION: return launch_stage3d_diffusion(stencil, tangent, kind, a, s);
    case RD_MODEL_BARKLEY: return launch_stage3d_barkley(stencil, tangent, kind, a, s);
    case RD_MODEL_FENTON_KARMA: return launch_stage3d_fk(stencil, tangent, kind, a, s);
    case RD_MODEL_BOCF: return launch_stage3d_bocf(stencil, tangent, kind, a, s);
    case RD_MODEL_FHN: return launch_stage3d_fhn(stencil, tangent, kind, a, s);
  }
  return hipErrorInvalidValue;
}

// The stage input coefficient a_s (Y_s = z + a_s k_{s-1}) and output weight B_s
// of stage s (0-based) of an explicit scheme with ns stages, as the forward
// forms them.
static double stage_a(const KConst& c, int ns, int st) { return st == 0 ? 0.0 : (ns == 4 && st < 3 ? c.h2 : c.dt); }
static double stage_b(const KConst& c, int ns, int st) {
  if (ns == 4) return st == 0 || st == 3 ? c.h6 : 2.0 * c.h6;
  return ns == 2 ? c.h2 : c.dt;
}

// The stage launches of one step from `zin` into `zout` (distinct arrays),
// storing k_1 .. k_{ns-1} in kb.  With `rates_only`, only those rates.
static int step_once_3d(const rd_problem* p, const KConst& c, bool tangent, double* const* zin, double* const* zout,
                        double* (*kb)[kMaxPacked3], const Stage3Args& base, hipStream_t s,
                        bool rates_only = false) {
  const int np = (tangent ? 2 : 1) * n_fields(p->model);
  const int ns = n_stages(p->scheme);
  const bool gate = gate_scheme(p->scheme);
  for (int st = 0; st < (rates_only ? ns - 1 : ns); ++st) {
    Stage3Args g = base;
    for (int f = 0; f < np; ++f) {
      // unused pointer slots point at valid arrays
      g.z[f] = zin[f];
      g.kp[f] = zin[f];
      g.kout[f] = zout ? zout[f] : zin[f];
      g.out[f] = zout ? zout[f] : zin[f];
      for (int j = 0; j < 3; ++j) g.ks[j][f] = zin[f];
    }
    int kind;
    const bool last = st == ns - 1;
    if (st > 0)
      for (int f = 0; f < np; ++f) g.kp[f] = kb[st - 1][f];
    g.a_in = stage_a(c, ns, st);
    if (!last) {
      kind = st == 0 ? kS3First : kS3Mid;
      for (int f = 0; f < np; ++f) g.kout[f] = kb[st][f];
    } else if (gate) {
      kind = p->scheme == RD_SCHEME_RUSH_LARSEN ? kS3GateRL : kS3GateIE;
    } else {
      kind = st == 0 ? kS3Final : kS3FinalKp;
      g.nk = ns - 1;
      for (int j = 0; j < ns - 1; ++j)
        for (int f = 0; f < np; ++f) g.ks[j][f] = kb[j][f];
      g.bw = ns == 4 ? c.h6 : (ns == 2 ? c.h2 : c.dt);
    }
    hipError_t e = launch_stage(p->model, p->stencil, tangent, kind, g, s);
    if (e != hipSuccess) return hip_fail(e, "3-D stage kernel launch");
  }
  return RD_OK;
}

size_t workspace_3d(const rd_problem* p, bool tangent) {
  const size_t np = (size_t)(tangent ? 2 : 1) * (size_t)n_fields(p->model);
  return (size_t)n_stages(p->scheme) * np * field_bytes(p);
}

// nsteps steps of the packed arrays `a` (NV state fields, then NV tangent
// fields when `tangent`), in place.  Workspace: the ping-pong state, then
// NS - 1 stored stage rates, each np fields of field_bytes(p).
int run_steps_3d(const rd_problem* p, const KConst& c, bool tangent, double* const* a, char* ws,
                 int64_t nsteps, double* checkpoints, int every, hipStream_t s) {
  const int nv = n_fields(p->model);
  const int np = tangent ? 2 * nv : nv;
  const int ns = n_stages(p->scheme);
  const size_t fb = field_bytes(p);
  const size_t cells = (size_t)p->nx * (size_t)p->ny * (size_t)p->nz;
  const size_t bytes = cells * sizeof(double);
  double* bufA[kMaxPacked3];
  double* bufB[kMaxPacked3];
  double* kb[3][kMaxPacked3];
  for (int f = 0; f < np; ++f) {
    bufA[f] = a[f];
    bufB[f] = (double*)(ws + (size_t)f * fb);
    for (int j = 0; j < ns - 1; ++j) kb[j][f] = (double*)(ws + ((size_t)(1 + j) * np + f) * fb);
  }
  double** cur = bufA;
  double** oth = bufB;
  if (nsteps % 2 == 1) {  // an odd number of steps must end in the caller's arrays
    int rc = copy_state(bufB, bufA, np, bytes, s);
    if (rc) return rc;
    cur = bufB;
    oth = bufA;
  }
  Stage3Args base;
  std::memset(&base, 0, sizeof base);
  base.c = c;
  geometry_3d(p, base);
  const bool ck = checkpoints && every > 0;

  for (int64_t n = 0; n < nsteps; ++n) {
    if (ck && n % every == 0) {
      double* dst[kMaxFields];
      for (int f = 0; f < nv; ++f) dst[f] = checkpoints + ((size_t)(n / every) * nv + f) * cells;
      int rc = copy_state(dst, cur, nv, bytes, s);
      if (rc) return rc;
    }
    int rc = step_once_3d(p, c, tangent, cur, oth, kb, base, s);
    if (rc) return rc;
    std::swap(cur, oth);
  }
  return RD_OK;
}

// Adjoint workspace: (C - 1) recomputed states, NS - 1 stage rates, two
// Ybar buffers, the running zbar and the cotangent's ping-pong partner, each
// n_fields arrays.
size_t workspace_vjp_3d(const rd_problem* p) {
  const size_t nv = (size_t)n_fields(p->model);
  const size_t C = (size_t)std::max(p->checkpoint_every, 1);
  return nv * ((C - 1) + (size_t)(n_stages(p->scheme) - 1) + 4) * field_bytes(p);
}

static hipError_t launch_adjoint3d(int model, int stencil, int kind, const Adj3Args& a, hipStream_t s) {
  switch (model) {
    case RD_MODEL_DIFFUSION: return launch_adjoint3d_diffusion(stencil, kind, a, s);
    case RD_MODEL_BARKLEY: return launch_adjoint3d_barkley(stencil, kind, a, s);
    case RD_MODEL_FENTON_KARMA: return launch_adjoint3d_fk(stencil, kind, a, s);
    case RD_MODEL_BOCF: return launch_adjoint3d_bocf(stencil, kind, a, s);
    case RD_MODEL_FHN: return launch_adjoint3d_fhn(stencil, kind, a, s);
  }
  return hipErrorInvalidValue;
}

// lambda_0 = (dPhi/dz_0)^T lambda_nsteps from the checkpoints of rd_step,
// segment by segment from the last: recompute the segment's states, then for
// each step backwards recompute its stage rates and run the reverse stages.
int vjp_3d(const rd_problem* p, const KConst& c, const double* checkpoints, double* const* cot, char* ws,
           hipStream_t s) {
  const int nv = n_fields(p->model);
  const int ns = n_stages(p->scheme);
  const int C = p->checkpoint_every;
  const size_t fb = field_bytes(p);
  const size_t cells = (size_t)p->nx * (size_t)p->ny * (size_t)p->nz;
  auto arr = [&](size_t i) { return (double*)(ws + i * fb); };
  const size_t o_k = (size_t)(C - 1) * nv, o_yb = o_k + (size_t)(ns - 1) * nv, o_zs = o_yb + 2 * (size_t)nv,
               o_lam = o_zs + nv;
  double* kb[3][kMaxPacked3];
  double* yb[2][kMaxFields];
  double* zs[kMaxFields];
  double* curA[kMaxFields];
  double* curB[kMaxFields];
  for (int f = 0; f < nv; ++f) {
    for (int j = 0; j < ns - 1; ++j) kb[j][f] = arr(o_k + (size_t)j * nv + f);
    yb[0][f] = arr(o_yb + f);
    yb[1][f] = arr(o_yb + nv + f);
    zs[f] = arr(o_zs + f);
    curA[f] = cot[f];
    curB[f] = arr(o_lam + f);
  }
  auto ckpt = [&](int64_t m, int f) { return (double*)checkpoints + ((size_t)m * nv + f) * cells; };
  auto seg_state = [&](int i, int f) { return arr((size_t)i * nv + f); };

  Stage3Args base;
  std::memset(&base, 0, sizeof base);
  base.c = c;
  geometry_3d(p, base);
  Adj3Args abase;
  std::memset(&abase, 0, sizeof abase);
  abase.c = c;
  geometry_3d(p, abase);

  double** cur = curA;
  double** oth = curB;
  if (p->nsteps % 2 == 1) {  // an odd number of swaps must end in the caller's arrays
    int rc = copy_state(curB, curA, nv, cells * sizeof(double), s);
    if (rc) return rc;
    std::swap(cur, oth);
  }
  const int64_t nck = (p->nsteps + C - 1) / C;
  for (int64_t m = nck - 1; m >= 0; --m) {
    const int64_t start = m * C;
    const int64_t stop = std::min(start + (int64_t)C, p->nsteps);
    auto state = [&](int64_t n, double** out) {
      for (int f = 0; f < nv; ++f) out[f] = n == start ? ckpt(m, f) : seg_state((int)(n - start - 1), f);
    };
    for (int64_t n = start + 1; n < stop; ++n) {  // recompute z_{start+1} .. z_{stop-1}
      double* zin[kMaxFields];
      double* zout[kMaxFields];
      state(n - 1, zin);
      state(n, zout);
      int rc = step_once_3d(p, c, false, zin, zout, kb, base, s);
      if (rc) return rc;
    }
    for (int64_t n = stop - 1; n >= start; --n) {
      double* z[kMaxFields];
      state(n, z);
      if (ns > 1) {
        int rc = step_once_3d(p, c, false, z, nullptr, kb, base, s, true);
        if (rc) return rc;
      }
      for (int j = ns - 1; j >= 0; --j) {  // reverse stage j (0-based)
        Adj3Args g = abase;
        for (int f = 0; f < nv; ++f) {
          g.z[f] = z[f];
          g.kp[f] = j > 0 ? kb[j - 1][f] : z[f];
          g.lam[f] = cur[f];
          g.yb_next[f] = j < ns - 1 ? yb[(j + 1) % 2][f] : cur[f];
          g.zs_in[f] = j == ns - 1 ? cur[f] : zs[f];
          g.zs_out[f] = j == 0 ? oth[f] : zs[f];
          g.yb_out[f] = yb[j % 2][f];
        }
        g.a_in = stage_a(c, ns, j);
        g.b_j = stage_b(c, ns, j);
        g.a_next = j < ns - 1 ? stage_a(c, ns, j + 1) : 0.0;
        const int kind = gate_scheme(p->scheme)
                             ? (p->scheme == RD_SCHEME_RUSH_LARSEN ? kA3GateRL : kA3GateIE)
                             : ns == 1 ? kA3Only : (j == ns - 1 ? kA3Last : (j == 0 ? kA3First : kA3Mid));
        hipError_t e = launch_adjoint3d(p->model, p->stencil, kind, g, s);
        if (e != hipSuccess) return hip_fail(e, "3-D adjoint stage launch");
      }
      std::swap(cur, oth);
    }
  }
  return RD_OK;
}

}  // namespace rd
