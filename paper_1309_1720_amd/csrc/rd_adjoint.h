// rd_adjoint.h -- one step of the discrete adjoint: lambda_n = (dPhi/dz_n)^T
// lambda_{n+1} for an explicit Euler / Heun / RK4 step.
//
// With stage inputs Y_s = z + a_s dt k_{s-1} and output z' = z + sum_s B_s k_s,
// the transposed step runs the stages backwards:
//   kbar_S = B_S lam;  for j = S .. 1:
//     Ybar_j = J(Y_j)^T kbar_j = (L^T kbar_j,u + J_N(Y_j)^T kbar_j)
//     kbar_{j-1} = B_{j-1} lam + a_j Ybar_j
//   lam_n = lam + Ybar_S + ... + Ybar_1.
// L is symmetric for the 5- and 9-point stencils with mirrored ghosts, so
// L^T kbar_u is the same stencil applied to kbar_u (for every diffusive
// field, each with its own diffusivity).  The anisotropic flux form is not
// symmetric; its transpose is applied in gather form (flux_transpose).  J_N(Y)^T comes from the
// reaction's Jacobian columns, evaluated on dual numbers.
//
// The gate schemes (one stage) transpose as lambda_n = J_P(z)^T lambda +
// dt L^T lambda_u, with P the step's pointwise part (gate_point_jt).
//
// The stage inputs Y_2 .. Y_S are produced beforehand by the stage-input mode
// of the sweep kernel (Y_1 = z_n).  This kernel uses the same decomposition
// as the sweep: one wavefront per 64-column strip and row band, halo NS, and
// reverse stage j running on row r - (NS - j + 1) while lambda row r loads.
#pragma once

#include "rd_sweep.h"

namespace rd {

struct AdjArgs {
  const double* z[kMaxFields];          // z_n
  const double* ys[3][kMaxFields];      // Y_2 .. Y_NS of the step from z_n
  const double* lam_in[kMaxFields];     // lambda_{n+1}
  double* lam_out[kMaxFields];          // lambda_n
  KConst c;
};

// out = J_N(y)^T a, column by column on dual numbers.
template <int MODEL>
__device__ __forceinline__ void reaction_jt(const KConst& c, const double* y, const double* a,
                                            double* out) {
  constexpr int NV = ModelTraits<MODEL>::NV;
#pragma unroll
  for (int l = 0; l < NV; ++l) {
    Dual yd[NV], kd[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) yd[f] = Dual(y[f], f == l ? 1.0 : 0.0);
    Reaction<MODEL>::template rates<Dual>(c, yd, kd);
    double acc = kd[0].d * a[0];
#pragma unroll
    for (int m = 1; m < NV; ++m) acc = acc + kd[m].d * a[m];
    out[l] = acc;
  }
}

// out = J_P(y)^T lam for the pointwise part P of a gate step (GATE 1:
// Rush-Larsen, 2: implicit Euler; gated models): the voltage's explicit
// Euler step on the reaction alone and each gate's update, differentiated
// column by column on dual numbers.  The diffusion term of the voltage is
// linear; its transpose (dt L^T lam_u) is added by the caller.
template <int MODEL, int GATE>
__device__ __forceinline__ void gate_point_jt(const KConst& c, const double* y, const double* lam,
                                              double* out) {
  constexpr int NV = ModelTraits<MODEL>::NV;
  static_assert(ModelTraits<MODEL>::GATED && ModelTraits<MODEL>::NDIFF == 1, "gated models only");
#pragma unroll
  for (int l = 0; l < NV; ++l) {
    Dual yd[NV], kd[NV], al[NV], be[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) yd[f] = Dual(y[f], f == l ? 1.0 : 0.0);
    Reaction<MODEL>::template rates<Dual>(c, yd, kd);
    Reaction<MODEL>::template gates<Dual>(c, yd, al, be);
    double acc = (yd[0] + c.dt * kd[0]).d * lam[0];
#pragma unroll
    for (int g = 1; g < NV; ++g) acc = acc + gate_step<GATE>(yd[g], al[g], be[g], c.dt).d * lam[g];
    out[l] = acc;
  }
}

// Cross-flux coefficients D_xy/4 at the centres of the west and east
// neighbour columns (the flux form's y-face terms reach them).
struct ColumnNb {
  double dxy_c4_w, dxy_c4_e;
};
__device__ __forceinline__ ColumnNb make_column_nb(int gx, const KConst& c) {
  const int gw = c.periodic ? wrap_index(gx - 1, c.nx) : gx - 1;
  const int ge = c.periodic ? wrap_index(gx + 1, c.nx) : gx + 1;
  const double thw = c.theta0 + c.dtheta * (((double)gw + 0.5) / c.n_total);
  const double the = c.theta0 + c.dtheta * (((double)ge + 0.5) / c.n_total);
  ColumnNb nb;
  nb.dxy_c4_w = 0.25 * ((c.dd * cos(thw)) * sin(thw));
  nb.dxy_c4_e = 0.25 * ((c.dd * cos(the)) * sin(the));
  return nb;
}

// (L^T a) at row J of this lane's column I for the anisotropic flux form
// L = s D G (G: cell values -> face fluxes, D: face fluxes -> cell
// divergence, zero flux through the boundary): with the face potentials
// psi_x(i, j) = a(i, j) - a(i+1, j) and psi_y(i, j) = a(i, j) - a(i, j+1)
// (= D^T a), every face flux formula scatters s psi times its coefficients
// back to the cells it reads; gathered here per cell, including the cells a
// mirrored (clamped) ghost index lands on.  up, cen, dn: a at rows J-1, J,
// J+1 (values outside the grid are not used).  All lanes call it together.
// YEDGE = false promises 0 < J < ny - 1 (the same operations, no y-face test).
template <bool EDGE, bool YEDGE = true>
__device__ __forceinline__ double flux_transpose(double up, double cen, double dn, const Column& col,
                                                 const ColumnNb& nb, int J, const KConst& c, double s) {
  const bool hasW = !(EDGE && col.west), hasE = !(EDGE && col.east);  // faces I-1/2, I+1/2 exist
  const bool atW = EDGE && col.west, atE = EDGE && col.east;          // I == 0, I == nx-1
  const bool hasU = !YEDGE || c.periodic || J >= 1, hasD = !YEDGE || c.periodic || J <= c.ny - 2;
  // x-face potentials of the east face at rows J-1, J, J+1, and of the west face
  const double pe_u = up - from_east(up), pe_c = cen - from_east(cen), pe_d = dn - from_east(dn);
  const double pw_u = from_west(pe_u), pw_c = from_west(pe_c), pw_d = from_west(pe_d);
  // y-face potentials of the faces above (J-1/2) and below (J+1/2), here and at I-1, I+1
  const double py_u = up - cen, py_d = cen - dn;
  const double pyw_u = from_west(py_u), pyw_d = from_west(py_d);
  const double pye_u = from_east(py_u), pye_d = from_east(py_d);

  double t = 0.0;
  // x-faces: the u(i+1, j) - u(i, j) term
  if (hasW) t += col.dxx_w * pw_c;
  if (hasE) t -= col.dxx_e * pe_c;
  // x-faces: cross terms (rows j+1 and j-1 of the face, clamped at the y-edges)
  auto cross_x = [&](double q, double pu, double pc, double pd) {
    double r = 0.0;
    if (hasU) r += q * pu;
    if (!hasD) r += q * pc;  // J == ny-1: the face's row j+1 is clamped to J
    if (hasD) r -= q * pd;
    if (!hasU) r -= q * pc;  // J == 0: the face's row j-1 is clamped to J
    return r;
  };
  if (hasW) t += cross_x(col.dxy_w4, pw_u, pw_c, pw_d);
  if (hasE) t += cross_x(col.dxy_e4, pe_u, pe_c, pe_d);
  // y-faces: the u(i, j+1) - u(i, j) term
  if (hasU) t += col.dyy_c * py_u;
  if (hasD) t -= col.dyy_c * py_d;
  // y-faces: cross terms, read at columns i+1 (clamped) and i-1 (clamped)
  auto cross_y = [&](double r, double pu, double pd) {
    double v = 0.0;
    if (hasU) v += r * pu;
    if (hasD) v += r * pd;
    return v;
  };
  if (hasW) t += cross_y(nb.dxy_c4_w, pyw_u, pyw_d);  // face of column I-1 reads I as its east column
  if (atE) t += cross_y(col.dxy_c4, py_u, py_d);      // I == nx-1: its own east column clamps to I
  if (hasE) t -= cross_y(nb.dxy_c4_e, pye_u, pye_d);  // face of column I+1 reads I as its west column
  if (atW) t -= cross_y(col.dxy_c4, py_u, py_d);      // I == 0: its own west column clamps to I
  return t * s;
}

template <int NS> struct AdjCoef;
template <> struct AdjCoef<1> {
  __device__ static double B(const KConst& c, int) { return c.dt; }
  __device__ static double A(const KConst&, int) { return 0.0; }
};
template <> struct AdjCoef<2> {
  __device__ static double B(const KConst& c, int) { return c.h2; }
  __device__ static double A(const KConst& c, int) { return c.dt; }
};
template <> struct AdjCoef<4> {
  // B = (dt/6, 2 dt/6, 2 dt/6, dt/6) as the forward applies them; a_j links
  // kbar_{j-1} to Ybar_j: a_2 = a_3 = dt/2, a_4 = dt.
  __device__ static double B(const KConst& c, int j) { return (j == 1 || j == 4) ? c.h6 : 2.0 * c.h6; }
  __device__ static double A(const KConst& c, int j) { return j == 4 ? c.dt : c.h2; }
};

// Register budget: two waves per SIMD, one for the four-variable model (its
// four dual-number Jacobian columns would spill otherwise).
template <int MODEL> struct AdjOccupancy { static constexpr int value = MODEL == RD_MODEL_BOCF ? 1 : 2; };

template <int MODEL, int STENCIL, int NS, int GATE = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(AdjOccupancy<MODEL>::value)))
void adjoint_kernel(AdjArgs a) {
  static_assert(GATE == 0 || NS == 1, "gate schemes have one stage");
  constexpr int NV = ModelTraits<MODEL>::NV;
  constexpr int NDF = ModelTraits<MODEL>::NDIFF;  // diffusive fields 0 .. NDF-1
  constexpr int TX = kWave - 2 * NS;
  constexpr int LR = (NS + 1 > 3) ? NS + 1 : 3;  // lambda rows kept: r .. r - LR + 1
  const KConst& c = a.c;

  const int lane = threadIdx.x & (kWave - 1);
  const int blk = xcd_order((int)blockIdx.x, (int)gridDim.x);
  const int wid = __builtin_amdgcn_readfirstlane(blk * (int)(blockDim.x / kWave) + (int)(threadIdx.x / kWave));
  if (wid >= c.nsx * c.nby) return;  // whole waves only: no barrier follows
  const int sx = wid / c.nby;  // bands of one strip are consecutive
  const int by = wid % c.nby;
  const int gx = sx * TX - NS + lane;
  const int cx = grid_index(gx, c.nx, c);
  const bool out_col = lane >= NS && lane < NS + TX && gx < c.nx;
  constexpr bool ANISO = STENCIL == RD_LAP9_ANISO;
  const Column col = make_column(gx, c, ANISO);
  const ColumnNb nb = ANISO ? make_column_nb(gx, c) : ColumnNb{0.0, 0.0};
  const bool edge = strip_touches_edge(sx * TX - NS, c);

  const int yA = by * c.ty;
  const int yB = min(yA + c.ty, c.ny);
  const int r_first = c.periodic ? yA - NS : max(yA - NS, 0);
  const int r_last = yB - 1 + NS;
  const int load_end = c.periodic ? yB + NS : min(yB + NS, c.ny);
  const size_t nx = (size_t)c.nx;

  double lr[LR][NV];          // lr[a] = lambda_{n+1} at row r - a
  double lacc[NS][NV];        // lacc[a] = running lambda_n at row r - 1 - a
  double kbu[NS + 1][3][NDF]; // kbar_j diffusive components at rows rho_j + 1, rho_j, rho_j - 1
  double kbg[NS + 1][NV];     // kbar_j other components at row rho_j
  double kbgn[NS + 1][NV];    // ... produced this iteration
#pragma unroll
  for (int k = 0; k < LR; ++k)
#pragma unroll
    for (int f = 0; f < NV; ++f) lr[k][f] = 0.0;
#pragma unroll
  for (int k = 0; k <= NS; ++k)
#pragma unroll
    for (int f = 0; f < NV; ++f) kbg[k][f] = kbgn[k][f] = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k)
#pragma unroll
    for (int f = 0; f < NV; ++f) lacc[k][f] = 0.0;
#pragma unroll
  for (int k = 0; k <= NS; ++k)
#pragma unroll
    for (int d = 0; d < NDF; ++d) kbu[k][0][d] = kbu[k][1][d] = kbu[k][2][d] = 0.0;

  double pre[NV];
#pragma unroll
  for (int f = 0; f < NV; ++f) pre[f] = 0.0;
  if (r_first < load_end) {
#pragma unroll
    for (int f = 0; f < NV; ++f) pre[f] = a.lam_in[f][(size_t)grid_index(r_first, c.ny, c) * nx + cx];
  }

  for (int r = r_first; r <= r_last; ++r) {
#pragma unroll
    for (int k = LR - 1; k > 0; --k)
#pragma unroll
      for (int f = 0; f < NV; ++f) lr[k][f] = lr[k - 1][f];
#pragma unroll
    for (int k = NS - 1; k > 0; --k)
#pragma unroll
      for (int f = 0; f < NV; ++f) lacc[k][f] = lacc[k - 1][f];
#pragma unroll
    for (int j = 1; j < NS; ++j) {
#pragma unroll
      for (int d = 0; d < NDF; ++d) {
        kbu[j][2][d] = kbu[j][1][d];
        kbu[j][1][d] = kbu[j][0][d];
      }
#pragma unroll
      for (int f = NDF; f < NV; ++f) kbg[j][f] = kbgn[j][f];
    }
    if (r < load_end) {
#pragma unroll
      for (int f = 0; f < NV; ++f) lr[0][f] = pre[f];
      if (r + 1 < load_end) {
        const size_t o = (size_t)grid_index(r + 1, c.ny, c) * nx + cx;
#pragma unroll
        for (int f = 0; f < NV; ++f) pre[f] = a.lam_in[f][o];
      }
    }

#pragma unroll
    for (int j = NS; j >= 1; --j) {
      const int lag = NS - j + 1;
      const int rho = r - lag;
      const int lo = c.periodic ? yA - (j - 1) : max(yA - (j - 1), 0);
      const int hi = c.periodic ? yB + (j - 1) : min(yB + (j - 1), c.ny);
      if (rho < lo || rho >= hi) continue;  // wave-uniform

      // kbar_j at rows rho-1, rho, rho+1 (diffusive fields) and rho (all)
      double kb[NV], up[NDF], dn[NDF];
      if (j == NS) {
        const double b = AdjCoef<NS>::B(c, j);
#pragma unroll
        for (int f = 0; f < NV; ++f) kb[f] = b * lr[lag][f];
#pragma unroll
        for (int d = 0; d < NDF; ++d) {
          up[d] = b * lr[lag + 1][d];
          dn[d] = b * lr[lag - 1][d];
        }
      } else {
#pragma unroll
        for (int d = 0; d < NDF; ++d) {
          kb[d] = kbu[j][1][d];
          up[d] = kbu[j][2][d];
          dn[d] = kbu[j][0][d];
        }
#pragma unroll
        for (int f = NDF; f < NV; ++f) kb[f] = kbg[j][f];
      }
      double lapT[NDF];
#pragma unroll
      for (int d = 0; d < NDF; ++d) {
        if (!c.periodic && rho == 0) up[d] = kb[d];
        if (!c.periodic && rho == c.ny - 1) dn[d] = kb[d];
        if constexpr (ANISO)
          lapT[d] = edge ? flux_transpose<true>(up[d], kb[d], dn[d], col, nb, rho, c, c.dcoef[d])
                         : flux_transpose<false>(up[d], kb[d], dn[d], col, nb, rho, c, c.dcoef[d]);
        else
          lapT[d] = edge ? diffusion<STENCIL, true>(up[d], kb[d], dn[d], col, rho, c, c.dcoef[d])
                         : diffusion<STENCIL, false>(up[d], kb[d], dn[d], col, rho, c, c.dcoef[d]);
      }

      double y[NV];
      const size_t o = (size_t)grid_index(rho, c.ny, c) * nx + cx;
      if (j == 1) {
#pragma unroll
        for (int f = 0; f < NV; ++f) y[f] = a.z[f][o];
      } else {
#pragma unroll
        for (int f = 0; f < NV; ++f) y[f] = a.ys[j - 2][f][o];
      }
      double yb[NV];
      if constexpr (GATE != 0) {
        // lambda_n = J_P^T lambda + L^T (dt lambda_u): the whole new value
        gate_point_jt<MODEL, GATE>(c, y, lr[lag], yb);
#pragma unroll
        for (int d = 0; d < NDF; ++d) yb[d] = yb[d] + lapT[d];
#pragma unroll
        for (int f = 0; f < NV; ++f) lacc[lag - 1][f] = yb[f];
      } else {
        reaction_jt<MODEL>(c, y, kb, yb);
#pragma unroll
        for (int d = 0; d < NDF; ++d) yb[d] = yb[d] + lapT[d];
      }

      if (GATE != 0) {
      } else if (j == NS) {
#pragma unroll
        for (int f = 0; f < NV; ++f) lacc[lag - 1][f] = lr[lag][f] + yb[f];
      } else {
#pragma unroll
        for (int f = 0; f < NV; ++f) lacc[lag - 1][f] = lacc[lag - 1][f] + yb[f];
      }
      if (j > 1) {
        const double b = AdjCoef<NS>::B(c, j - 1);
        const double aj = AdjCoef<NS>::A(c, j);
#pragma unroll
        for (int d = 0; d < NDF; ++d) kbu[j - 1][0][d] = b * lr[lag][d] + aj * yb[d];
#pragma unroll
        for (int f = NDF; f < NV; ++f) kbgn[j - 1][f] = b * lr[lag][f] + aj * yb[f];
      } else if (out_col && rho >= yA && rho < yB) {
        const size_t oo = (size_t)rho * nx + gx;
#pragma unroll
        for (int f = 0; f < NV; ++f) a.lam_out[f][oo] = lacc[lag - 1][f];
      }
    }
  }
}

template <int MODEL, int STENCIL, int NS, int GATE = 0>
hipError_t launch_adjoint(const AdjArgs& a, hipStream_t stream) {
  const int waves = a.c.nsx * a.c.nby;
  const int blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((adjoint_kernel<MODEL, STENCIL, NS, GATE>), dim3(blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

// The gate schemes' adjoint (one stage; gated models only).
template <int MODEL, int STENCIL>
hipError_t launch_adjoint_gate(int scheme, const AdjArgs& a, hipStream_t s) {
  if constexpr (ModelTraits<MODEL>::GATED) {
    if (scheme == RD_SCHEME_RUSH_LARSEN) return launch_adjoint<MODEL, STENCIL, 1, 1>(a, s);
    if (scheme == RD_SCHEME_IMPLICIT_EULER) return launch_adjoint<MODEL, STENCIL, 1, 2>(a, s);
  }
  return hipErrorInvalidValue;
}

template <int MODEL>
hipError_t launch_adjoint_model(int stencil, int scheme, const AdjArgs& a, hipStream_t s) {
  switch (stencil) {
    case RD_LAP5:
      if (scheme == RD_SCHEME_EULER) return launch_adjoint<MODEL, RD_LAP5, 1>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_adjoint<MODEL, RD_LAP5, 2>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_adjoint<MODEL, RD_LAP5, 4>(a, s);
      return launch_adjoint_gate<MODEL, RD_LAP5>(scheme, a, s);
    case RD_LAP9:
      if (scheme == RD_SCHEME_EULER) return launch_adjoint<MODEL, RD_LAP9, 1>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_adjoint<MODEL, RD_LAP9, 2>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_adjoint<MODEL, RD_LAP9, 4>(a, s);
      return launch_adjoint_gate<MODEL, RD_LAP9>(scheme, a, s);
    case RD_LAP9_ANISO:
      if (scheme == RD_SCHEME_EULER) return launch_adjoint<MODEL, RD_LAP9_ANISO, 1>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_adjoint<MODEL, RD_LAP9_ANISO, 2>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_adjoint<MODEL, RD_LAP9_ANISO, 4>(a, s);
      return launch_adjoint_gate<MODEL, RD_LAP9_ANISO>(scheme, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint_diffusion(int stencil, int scheme, const AdjArgs& a, hipStream_t s);
hipError_t launch_adjoint_barkley(int stencil, int scheme, const AdjArgs& a, hipStream_t s);
hipError_t launch_adjoint_fk(int stencil, int scheme, const AdjArgs& a, hipStream_t s);
hipError_t launch_adjoint_bocf(int stencil, int scheme, const AdjArgs& a, hipStream_t s);
hipError_t launch_adjoint_fhn(int stencil, int scheme, const AdjArgs& a, hipStream_t s);

}  // namespace rd
