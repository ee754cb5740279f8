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
// field, each with its own diffusivity).  J_N(Y)^T comes from the
// reaction's Jacobian columns, evaluated on dual numbers.
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

template <int MODEL, int STENCIL, int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(AdjOccupancy<MODEL>::value)))
void adjoint_kernel(AdjArgs a) {
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
  const int cx = min(max(gx, 0), c.nx - 1);
  const bool out_col = lane >= NS && lane < NS + TX && gx < c.nx;
  const Column col = make_column(gx, c, false);
  const bool edge = strip_touches_edge(sx * TX - NS, c);

  const int yA = by * c.ty;
  const int yB = min(yA + c.ty, c.ny);
  const int r_first = max(yA - NS, 0);
  const int r_last = yB - 1 + NS;
  const int load_end = min(yB + NS, c.ny);
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
    for (int f = 0; f < NV; ++f) pre[f] = a.lam_in[f][(size_t)r_first * nx + cx];
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
        const size_t o = (size_t)(r + 1) * nx + cx;
#pragma unroll
        for (int f = 0; f < NV; ++f) pre[f] = a.lam_in[f][o];
      }
    }

#pragma unroll
    for (int j = NS; j >= 1; --j) {
      const int lag = NS - j + 1;
      const int rho = r - lag;
      const int lo = max(yA - (j - 1), 0);
      const int hi = min(yB + (j - 1), c.ny);
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
        if (rho == 0) up[d] = kb[d];
        if (rho == c.ny - 1) dn[d] = kb[d];
        lapT[d] = edge ? diffusion<STENCIL, true>(up[d], kb[d], dn[d], col, rho, c, c.dcoef[d])
                       : diffusion<STENCIL, false>(up[d], kb[d], dn[d], col, rho, c, c.dcoef[d]);
      }

      double y[NV];
      const size_t o = (size_t)rho * nx + cx;
      if (j == 1) {
#pragma unroll
        for (int f = 0; f < NV; ++f) y[f] = a.z[f][o];
      } else {
#pragma unroll
        for (int f = 0; f < NV; ++f) y[f] = a.ys[j - 2][f][o];
      }
      double yb[NV];
      reaction_jt<MODEL>(c, y, kb, yb);
#pragma unroll
      for (int d = 0; d < NDF; ++d) yb[d] = yb[d] + lapT[d];

      if (j == NS) {
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

template <int MODEL, int STENCIL, int NS>
hipError_t launch_adjoint(const AdjArgs& a, hipStream_t stream) {
  const int waves = a.c.nsx * a.c.nby;
  const int blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((adjoint_kernel<MODEL, STENCIL, NS>), dim3(blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

template <int MODEL>
hipError_t launch_adjoint_model(int stencil, int scheme, const AdjArgs& a, hipStream_t s) {
  switch (stencil) {
    case RD_LAP5:
      if (scheme == RD_SCHEME_EULER) return launch_adjoint<MODEL, RD_LAP5, 1>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_adjoint<MODEL, RD_LAP5, 2>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_adjoint<MODEL, RD_LAP5, 4>(a, s);
      break;
    case RD_LAP9:
      if (scheme == RD_SCHEME_EULER) return launch_adjoint<MODEL, RD_LAP9, 1>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_adjoint<MODEL, RD_LAP9, 2>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_adjoint<MODEL, RD_LAP9, 4>(a, s);
      break;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint_diffusion(int stencil, int scheme, const AdjArgs& a, hipStream_t s);
hipError_t launch_adjoint_barkley(int stencil, int scheme, const AdjArgs& a, hipStream_t s);
hipError_t launch_adjoint_fk(int stencil, int scheme, const AdjArgs& a, hipStream_t s);
hipError_t launch_adjoint_bocf(int stencil, int scheme, const AdjArgs& a, hipStream_t s);
hipError_t launch_adjoint_fhn(int stencil, int scheme, const AdjArgs& a, hipStream_t s);

}  // namespace rd
