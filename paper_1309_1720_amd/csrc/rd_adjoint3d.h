// rd_adjoint3d.h -- one reverse stage of the discrete adjoint on a 3-D grid
// (the 7/19/27-point operators of rd_stage3d.h).
//
// For stage inputs Y_j = z + a_j k_{j-1} and output z' = z + sum_j B_j k_j,
// the transposed step runs the stages backwards from zbar = lambda:
//   kbar_j = B_j lambda + a_{j+1} Ybar_{j+1}      (no second term for j = S)
//   Ybar_j = J_N(Y_j)^T kbar_j + L kbar_j          (L on the diffusive fields)
//   zbar  += Ybar_j,
// and lambda_n = zbar after j = 1 (a gate step: lambda_n = J_P(z)^T lambda +
// dt L lambda_u, P its pointwise part).  The 3-D operators are symmetric under
// both boundary rules (mirrored ghosts, periodic wrap), so L^T = L.  Y_j is a
// pointwise input (the reaction's Jacobian); the operator acts on kbar_j,
// which is formed at the neighbour rows from lambda and Ybar_{j+1} while the
// plane is loaded -- the same plane ring and aligned 64-column strips as the
// forward stage kernel.  One launch per reverse stage; each streams its
// operands once (HBM-bound).
#pragma once

#include "rd_adjoint.h"
#include "rd_stage3d.h"

namespace rd {

struct Adj3Args {
  KConst c;
  int nz, zc, nbx, nby, nbz;
  const double* z[kMaxFields];        // z_n
  const double* kp[kMaxFields];       // k_{j-1} (HASKP): Y_j = z + a_in kp
  double a_in;
  const double* lam[kMaxFields];      // lambda_{n+1}
  double b_j;                         // B_j
  const double* yb_next[kMaxFields];  // Ybar_{j+1} (HASYB)
  double a_next;                      // a_{j+1}
  const double* zs_in[kMaxFields];    // running zbar (lambda for j = S)
  double* zs_out[kMaxFields];         // zbar + Ybar_j (lambda_n after j = 1); may alias zs_in
  double* yb_out[kMaxFields];         // Ybar_j (WRITEYB)
};

template <int MODEL, int STENCIL, bool HASKP, bool HASYB, bool WRITEYB, int GATE = 0>
__global__ __launch_bounds__(kStage3Waves* kWave) void adjoint3d_kernel(Adj3Args a) {
  static_assert(GATE == 0 || (!HASKP && !HASYB && !WRITEYB), "gate schemes have one stage");
  constexpr int NV = ModelTraits<MODEL>::NV;
  constexpr int ND = ModelTraits<MODEL>::NDIFF;
  constexpr bool DIAG = STENCIL != RD_LAP7;
  using W = Weights3<STENCIL>;
  const KConst& c = a.c;

  const int nblk = a.nbx * a.nby * a.nbz;
  const int b = xcd_order((int)blockIdx.x, nblk);
  const int by = b % a.nby;
  const int bz = (b / a.nby) % a.nbz;
  const int bx = b / (a.nby * a.nbz);
  const int lane = threadIdx.x & (kWave - 1);
  const int gy = by * kStage3Waves + (int)(threadIdx.x >> 6);
  if (gy >= c.ny) return;  // whole wavefront
  const int gx = bx * kStage3Width + lane;
  const bool out_col = gx < c.nx;
  const bool edge = lane == 0 || lane == kWave - 1;
  const size_t hx = (size_t)grid_index(lane == 0 ? bx * kStage3Width - 1 : bx * kStage3Width + kWave, c.nx, c);
  const size_t nx = (size_t)c.nx;
  const size_t plane = nx * (size_t)c.ny;
  const size_t cx = (size_t)grid_index(gx, c.nx, c);
  const size_t rowN = (size_t)grid_index(gy - 1, c.ny, c) * nx, rowS = (size_t)grid_index(gy + 1, c.ny, c) * nx;
  const size_t rC = (size_t)gy * nx + cx, rN = rowN + cx, rS = rowS + cx;
  const size_t hC = (size_t)gy * nx + hx, hN = rowN + hx, hS = rowS + hx;

  // kbar_j of field f at offset o
  auto kbar = [&](int f, size_t o) -> double {
    if constexpr (HASYB) return a.b_j * a.lam[f][o] + a.a_next * a.yb_next[f][o];
    return a.b_j * a.lam[f][o];
  };
  auto west = [&](double v, double h) {
    const double w = from_west(v);
    return lane == 0 ? h : w;
  };
  auto east = [&](double v, double h) {
    const double e = from_east(v);
    return lane == kWave - 1 ? h : e;
  };

  double U[3][ND], F[3][ND], G[3][ND];
  auto load_plane = [&](int pz, int slot) {
    const size_t base = (size_t)grid_index(pz, a.nz, c) * plane;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double vc = kbar(d, base + rC), vn = kbar(d, base + rN), vs = kbar(d, base + rS);
      double hc = 0.0, hn = 0.0, hs = 0.0;
      if (edge) {
        hc = kbar(d, base + hC);
        hn = kbar(d, base + hN);
        hs = kbar(d, base + hS);
      }
      const double cs = vn + vs;
      U[slot][d] = vc;
      F[slot][d] = (west(vc, hc) + east(vc, hc)) + cs;
      if constexpr (DIAG) G[slot][d] = west(cs, hn + hs) + east(cs, hn + hs);
    }
  };

  const int z0 = bz * a.zc;
  const int z1 = min(z0 + a.zc, a.nz);
  load_plane(z0 - 1, 0);
  load_plane(z0, 1);
  for (int pz = z0; pz < z1; ++pz) {
    load_plane(pz + 1, 2);
    const size_t o = (size_t)pz * plane + rC;
    double y[NV], kb[NV], yb[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) {
      if constexpr (HASKP) y[f] = a.z[f][o] + a.a_in * a.kp[f][o];
      else y[f] = a.z[f][o];
      kb[f] = kbar(f, o);
    }
    if constexpr (GATE != 0) {
      // gate step: lambda_n = J_P(z)^T lambda + L (dt lambda_u), the whole new value
      double lam_c[NV];
#pragma unroll
      for (int f = 0; f < NV; ++f) lam_c[f] = a.lam[f][o];
      gate_point_jt<MODEL, GATE>(c, y, lam_c, yb);
    } else {
      reaction_jt<MODEL>(c, y, kb, yb);
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double cen = U[1][d];
      const double faces = F[1][d] + (U[0][d] + U[2][d]);
      double s = W::f * (faces - 6.0 * cen);
      if constexpr (W::e != 0.0) {
        const double edges = G[1][d] + (F[0][d] + F[2][d]);
        s = s + W::e * (edges - 12.0 * cen);
      }
      if constexpr (W::c != 0.0) {
        const double corners = G[0][d] + G[2][d];
        s = s + W::c * (corners - 8.0 * cen);
      }
      yb[d] = yb[d] + c.dcoef[d] * s;
    }
    if (out_col) {
#pragma unroll
      for (int f = 0; f < NV; ++f) {
        const double zs = GATE != 0 ? 0.0 : a.zs_in[f][o];
        __builtin_nontemporal_store(GATE != 0 ? yb[f] : zs + yb[f], &a.zs_out[f][o]);
        if constexpr (WRITEYB) __builtin_nontemporal_store(yb[f], &a.yb_out[f][o]);
      }
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      U[0][d] = U[1][d];
      U[1][d] = U[2][d];
      F[0][d] = F[1][d];
      F[1][d] = F[2][d];
      if constexpr (DIAG) {
        G[0][d] = G[1][d];
        G[1][d] = G[2][d];
      }
    }
  }
}

// Reverse-stage kinds: the last stage (no Ybar_{j+1}), middle stages, the
// first stage of a multi-stage scheme (no k_0, no Ybar output), and Euler's
// only stage.
enum Adj3Kind { kA3Last = 0, kA3Mid = 1, kA3First = 2, kA3Only = 3, kA3GateRL = 4, kA3GateIE = 5 };

template <int MODEL, int STENCIL>
hipError_t launch_adjoint3d_st(int kind, const Adj3Args& a, hipStream_t s) {
  const dim3 grid((unsigned)(a.nbx * a.nby * a.nbz)), block(kStage3Waves * kWave);
  switch (kind) {
    case kA3Last: hipLaunchKernelGGL((adjoint3d_kernel<MODEL, STENCIL, true, false, true>), grid, block, 0, s, a); break;
    case kA3Mid: hipLaunchKernelGGL((adjoint3d_kernel<MODEL, STENCIL, true, true, true>), grid, block, 0, s, a); break;
    case kA3First: hipLaunchKernelGGL((adjoint3d_kernel<MODEL, STENCIL, false, true, false>), grid, block, 0, s, a); break;
    case kA3Only: hipLaunchKernelGGL((adjoint3d_kernel<MODEL, STENCIL, false, false, false>), grid, block, 0, s, a); break;
    case kA3GateRL:
    case kA3GateIE:
      if constexpr (ModelTraits<MODEL>::GATED) {
        if (kind == kA3GateRL)
          hipLaunchKernelGGL((adjoint3d_kernel<MODEL, STENCIL, false, false, false, 1>), grid, block, 0, s, a);
        else
          hipLaunchKernelGGL((adjoint3d_kernel<MODEL, STENCIL, false, false, false, 2>), grid, block, 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODEL>
hipError_t launch_adjoint3d_model(int stencil, int kind, const Adj3Args& a, hipStream_t s) {
  switch (stencil) {
    case RD_LAP7: return launch_adjoint3d_st<MODEL, RD_LAP7>(kind, a, s);
    case RD_LAP19: return launch_adjoint3d_st<MODEL, RD_LAP19>(kind, a, s);
    case RD_LAP27: return launch_adjoint3d_st<MODEL, RD_LAP27>(kind, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint3d_diffusion(int stencil, int kind, const Adj3Args& a, hipStream_t s);
hipError_t launch_adjoint3d_barkley(int stencil, int kind, const Adj3Args& a, hipStream_t s);
hipError_t launch_adjoint3d_fk(int stencil, int kind, const Adj3Args& a, hipStream_t s);
hipError_t launch_adjoint3d_bocf(int stencil, int kind, const Adj3Args& a, hipStream_t s);
hipError_t launch_adjoint3d_fhn(int stencil, int kind, const Adj3Args& a, hipStream_t s);

}  // namespace rd
