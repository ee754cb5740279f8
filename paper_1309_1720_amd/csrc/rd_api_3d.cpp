// rd_api_3d.cpp -- host side of the 3-D stencils: launch geometry, workspace
// layout and the stage sequence of each scheme (rd_stage3d.h).
#include <algorithm>
#include <cstring>

#include "rd_host.h"
#include "rd_stage3d.h"

namespace rd {

bool is_3d(int stencil) { return stencil == RD_LAP7 || stencil == RD_LAP19 || stencil == RD_LAP27; }

// Workgroup grid: 64-column strips x groups of four rows x chunks of zc
// planes, with enough chunks for about 8192 wavefronts (32 per CU) and at
// least four planes per chunk (each chunk reads two extra planes).
static void geometry_3d(const rd_problem* p, Stage3Args& a) {
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
  const bool gate = gate_scheme(p->scheme);

  for (int64_t n = 0; n < nsteps; ++n) {
    if (ck && n % every == 0) {
      double* dst[kMaxFields];
      for (int f = 0; f < nv; ++f) dst[f] = checkpoints + ((size_t)(n / every) * nv + f) * cells;
      int rc = copy_state(dst, cur, nv, bytes, s);
      if (rc) return rc;
    }
    // stage s of ns: input z (+ a_in k_{s-1}); output k_s, or the new state
    for (int st = 0; st < ns; ++st) {
      Stage3Args g = base;
      for (int f = 0; f < np; ++f) {
        // unused pointer slots point at valid arrays
        g.z[f] = cur[f];
        g.kp[f] = cur[f];
        g.kout[f] = oth[f];
        g.out[f] = oth[f];
        for (int j = 0; j < 3; ++j) g.ks[j][f] = cur[f];
      }
      int kind;
      const bool last = st == ns - 1;
      if (st > 0)
        for (int f = 0; f < np; ++f) g.kp[f] = kb[st - 1][f];
      g.a_in = st == 0 ? 0.0 : (ns == 4 && st < 3 ? c.h2 : c.dt);
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
    std::swap(cur, oth);
  }
  return RD_OK;
}

}  // namespace rd
