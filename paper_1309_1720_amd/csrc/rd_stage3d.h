// rd_stage3d.h -- one explicit stage on a 3-D grid (the 7/19/27-point
// operators; the paper's conclusion anticipates 3-D tissue and gives no 3-D
// stencil).
//
// Design.  Each launch evaluates one stage of the scheme (Sect. 4: diffusion,
// then reaction, then the Euler-like update) for the whole grid; stages that
// feed a later one store their rate k_s, the last stage combines the stored
// rates into the new state.  Fusing the stages of a step into one launch, as
// the 2-D sweep does, would need halos recomputed in x and y at once (a
// stage's neighbours in both directions belong to other wavefronts); with
// four RK4 stages that leaves well under two thirds of the lanes useful, so
// the unfused form, which streams its operands once per stage, is as fast
// and much simpler.  Each launch is HBM-bound.
//
// Geometry.  A workgroup is four wavefronts; wavefront w holds row y0 + w of
// a 64-column strip aligned to 64 columns (every lane an output; the
// x-neighbours come from the adjacent lanes through DPP, and lanes 0 and 63
// fetch the one column beyond each end of the strip in an extra load) and
// marches through a chunk of zc planes.  Aligned strips keep every row
// access and every store on whole cache lines; strips with halo lanes
// (62 outputs starting one column early) split each access across an extra
// line and were measured about 25% slower.  Results are written with
// nontemporal stores (streamed out, read again only by a later launch):
// 2-5% faster than plain stores on the stage kernels.  Per plane and diffusive component it loads rows y - 1, y, y + 1
// and forms three aggregates: U (the cell), F (its four in-plane face
// neighbours) and G (its four in-plane diagonals).  A register ring keeps
// them for planes z - 1, z, z + 1, from which the 26-neighbour groups follow:
//   faces   = F(z) + (U(z-1) + U(z+1))
//   edges   = G(z) + (F(z-1) + F(z+1))
//   corners = G(z-1) + G(z+1).
// Out-of-grid neighbours are read at clamped indices (no-flux: the mirror
// ghost of a reach-one stencil is the boundary cell itself, Fig. 1, in every
// direction, corners included) or wrapped ones (periodic).
#pragma once

#include "rd_device.h"

namespace rd {

constexpr int kStage3Waves = 4;              // rows (wavefronts) per workgroup
constexpr int kStage3Width = kWave;          // output columns per wavefront
constexpr int kMaxPacked3 = 2 * kMaxFields;  // state fields, then tangent fields

// 3-D stencil weights (faces, edges, corners); see include/rd.h.
template <int STENCIL> struct Weights3;
template <> struct Weights3<RD_LAP7> {
  static constexpr double f = 1.0, e = 0.0, c = 0.0;
};
template <> struct Weights3<RD_LAP19> {
  static constexpr double f = 1.0 / 3.0, e = 1.0 / 6.0, c = 0.0;
};
template <> struct Weights3<RD_LAP27> {
  static constexpr double f = 7.0 / 15.0, e = 1.0 / 10.0, c = 1.0 / 30.0;
};

struct Stage3Args {
  KConst c;
  int nz, zc;                              // planes; planes per workgroup chunk
  int nbx, nby, nbz;                       // workgroup grid (strips, row groups, chunks)
  const double* z[kMaxPacked3];            // state at the start of the step
  const double* kp[kMaxPacked3];           // previous stage rate (HASKP)
  double a_in;                             // stage input Y = z + a_in kp
  double* kout[kMaxPacked3];               // this stage's rate (not FINAL)
  const double* ks[3][kMaxPacked3];        // stored rates k_1 .. k_nk (FINAL)
  int nk;                                  // 0 (Euler), 1 (Heun), 3 (RK4)
  double bw;                               // z' = z + bw (k_1 + 2 k_2 + 2 k_3 + k_now)
  double* out[kMaxPacked3];                // new state (FINAL)
};

// HASKP: the stage input adds a_in times the previous rate.  FINAL: combine
// into the new state (GATE 1/2: Rush-Larsen / implicit-Euler gates) instead
// of storing the rate.  TAN: carry the tangent fields with dual numbers.
template <int MODEL, int STENCIL, bool TAN, bool HASKP, bool FINAL, int GATE>
__global__ __launch_bounds__(kStage3Waves* kWave) void stage3d_kernel(Stage3Args a) {
  constexpr int NV = ModelTraits<MODEL>::NV;
  constexpr int NDF = ModelTraits<MODEL>::NDIFF;
  constexpr int NF = TAN ? 2 * NV : NV;
  constexpr int ND = TAN ? 2 * NDF : NDF;
  constexpr bool DIAG = STENCIL != RD_LAP7;
  using W = Weights3<STENCIL>;
  static_assert(GATE == 0 || (FINAL && !HASKP), "gate schemes have one stage");
  auto comp = [](int d) { return d < NDF ? d : NV + (d - NDF); };
  const KConst& c = a.c;

  const int nblk = a.nbx * a.nby * a.nbz;
  const int b = xcd_order((int)blockIdx.x, nblk);
  const int by = b % a.nby;  // row groups of one strip and chunk are consecutive
  const int bz = (b / a.nby) % a.nbz;
  const int bx = b / (a.nby * a.nbz);
  const int lane = threadIdx.x & (kWave - 1);
  const int gy = by * kStage3Waves + (int)(threadIdx.x >> 6);
  if (gy >= c.ny) return;  // whole wavefront
  const int gx = bx * kStage3Width + lane;
  const bool out_col = gx < c.nx;
  const bool edge = lane == 0 || lane == kWave - 1;
  // lane 0 fetches the column west of the strip, lane 63 the one east of it
  const size_t hx = (size_t)grid_index(lane == 0 ? bx * kStage3Width - 1 : bx * kStage3Width + kWave, c.nx, c);
  const size_t nx = (size_t)c.nx;
  const size_t plane = nx * (size_t)c.ny;
  const size_t cx = (size_t)grid_index(gx, c.nx, c);
  const size_t rC = (size_t)gy * nx + cx;
  const size_t rN = (size_t)grid_index(gy - 1, c.ny, c) * nx + cx;
  const size_t rS = (size_t)grid_index(gy + 1, c.ny, c) * nx + cx;
  const size_t hC = (size_t)gy * nx + hx;
  const size_t hN = (size_t)grid_index(gy - 1, c.ny, c) * nx + hx;
  const size_t hS = (size_t)grid_index(gy + 1, c.ny, c) * nx + hx;

  auto yval = [&](int f, size_t o) -> double {
    if constexpr (HASKP) return a.z[f][o] + a.a_in * a.kp[f][o];
    return a.z[f][o];
  };

  // x-neighbours: the adjacent lane's value, or the fetched one past the strip
  auto west = [&](double v, double h) {
    const double w = from_west(v);
    return lane == 0 ? h : w;
  };
  auto east = [&](double v, double h) {
    const double e = from_east(v);
    return lane == kWave - 1 ? h : e;
  };

  // ring slot 0/1/2 = planes z-1, z, z+1
  double U[3][ND], F[3][ND], G[3][ND];
  auto load_plane = [&](int pz, int slot) {
    const size_t base = (size_t)grid_index(pz, a.nz, c) * plane;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const int f = comp(d);
      const double yc = yval(f, base + rC), yn = yval(f, base + rN), ys = yval(f, base + rS);
      double hc = 0.0, hn = 0.0, hs = 0.0;
      if (edge) {
        hc = yval(f, base + hC);
        hn = yval(f, base + hN);
        hs = yval(f, base + hS);
      }
      // the in-plane diagonals are the x-neighbours' N + S: one exchange
      const double cs = yn + ys;
      U[slot][d] = yc;
      F[slot][d] = (west(yc, hc) + east(yc, hc)) + cs;
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
    double zc_[NF], y[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      zc_[f] = a.z[f][o];
      if constexpr (HASKP) y[f] = zc_[f] + a.a_in * a.kp[f][o];
      else y[f] = zc_[f];
    }
    double kr[NF];
    eval_rates<MODEL, TAN>(c, y, kr);
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
      const int f = comp(d);
      kr[f] = c.dcoef[d % NDF] * s + kr[f];
    }
    if (out_col) {
      if constexpr (!FINAL) {
#pragma unroll
        for (int f = 0; f < NF; ++f) __builtin_nontemporal_store(kr[f], &a.kout[f][o]);
      } else if constexpr (GATE != 0) {
        double zn[NF];
        gate_scheme_step<MODEL, TAN, GATE>(c, y, kr, zn);
#pragma unroll
        for (int f = 0; f < NF; ++f) __builtin_nontemporal_store(zn[f], &a.out[f][o]);
      } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          double acc = kr[f];
          if (a.nk > 0) {
            acc = a.ks[0][f][o];
#pragma unroll
            for (int j = 1; j < 3; ++j)
              if (j < a.nk) acc = acc + 2.0 * a.ks[j][f][o];
            acc = acc + kr[f];
          }
          __builtin_nontemporal_store(zc_[f] + a.bw * acc, &a.out[f][o]);
        }
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

// Stage kinds of one step (host order): first stage (Y = z), middle stages
// (Y = z + a kp), last stage with or without a previous rate, gate step.
enum Stage3Kind { kS3First = 0, kS3Mid = 1, kS3Final = 2, kS3FinalKp = 3, kS3GateRL = 4, kS3GateIE = 5 };

template <int MODEL, int STENCIL, bool TAN>
hipError_t launch_stage3d_st(int kind, const Stage3Args& a, hipStream_t s) {
  const dim3 grid((unsigned)(a.nbx * a.nby * a.nbz)), block(kStage3Waves * kWave);
  switch (kind) {
    case kS3First: hipLaunchKernelGGL((stage3d_kernel<MODEL, STENCIL, TAN, false, false, 0>), grid, block, 0, s, a); break;
    case kS3Mid: hipLaunchKernelGGL((stage3d_kernel<MODEL, STENCIL, TAN, true, false, 0>), grid, block, 0, s, a); break;
    case kS3Final: hipLaunchKernelGGL((stage3d_kernel<MODEL, STENCIL, TAN, false, true, 0>), grid, block, 0, s, a); break;
    case kS3FinalKp: hipLaunchKernelGGL((stage3d_kernel<MODEL, STENCIL, TAN, true, true, 0>), grid, block, 0, s, a); break;
    case kS3GateRL:
    case kS3GateIE:
      if constexpr (ModelTraits<MODEL>::GATED) {
        if (kind == kS3GateRL)
          hipLaunchKernelGGL((stage3d_kernel<MODEL, STENCIL, TAN, false, true, 1>), grid, block, 0, s, a);
        else
          hipLaunchKernelGGL((stage3d_kernel<MODEL, STENCIL, TAN, false, true, 2>), grid, block, 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODEL>
hipError_t launch_stage3d_model(int stencil, bool tangent, int kind, const Stage3Args& a, hipStream_t s) {
  switch (stencil) {
    case RD_LAP7: return tangent ? launch_stage3d_st<MODEL, RD_LAP7, true>(kind, a, s) : launch_stage3d_st<MODEL, RD_LAP7, false>(kind, a, s);
    case RD_LAP19: return tangent ? launch_stage3d_st<MODEL, RD_LAP19, true>(kind, a, s) : launch_stage3d_st<MODEL, RD_LAP19, false>(kind, a, s);
    case RD_LAP27: return tangent ? launch_stage3d_st<MODEL, RD_LAP27, true>(kind, a, s) : launch_stage3d_st<MODEL, RD_LAP27, false>(kind, a, s);
  }
  return hipErrorInvalidValue;
}

// Per-model entry points (one translation unit each).
hipError_t launch_stage3d_diffusion(int stencil, bool tangent, int kind, const Stage3Args& a, hipStream_t s);
hipError_t launch_stage3d_barkley(int stencil, bool tangent, int kind, const Stage3Args& a, hipStream_t s);
hipError_t launch_stage3d_fk(int stencil, bool tangent, int kind, const Stage3Args& a, hipStream_t s);
hipError_t launch_stage3d_bocf(int stencil, bool tangent, int kind, const Stage3Args& a, hipStream_t s);
hipError_t launch_stage3d_fhn(int stencil, bool tangent, int kind, const Stage3Args& a, hipStream_t s);

}  // namespace rd
