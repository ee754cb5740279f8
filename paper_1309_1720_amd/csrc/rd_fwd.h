// rd_fwd.h -- fused explicit step: every stage of one Euler / Heun / RK4 step
// (stencil, reaction and Euler-like update, Sect. 4) in a single kernel.
//
// Work decomposition.  A wavefront owns a strip of 64 consecutive columns and
// a band of `ty` rows.  Its lanes hold one column each; a step of NS stages
// needs NS halo columns on either side, so a strip produces TX = 64 - 2 NS
// output columns.  The wave sweeps down its band one row per iteration: at
// iteration r it loads row r of the state and runs stage s on row r - s, so
// the three rows each stage's stencil needs are already in registers (rows
// r-s+1 .. r-s-1 of the previous stage's output) and the per-row state (z_n,
// the stage sum, the gate values of the stage input) lives in small register
// rings.  Each cell of the state is read once and written once per step;
// the only redundant work is the NS halo columns and the NS-row ramp at the
// ends of each band.  x-neighbours come from adjacent lanes (shuffles), so
// no LDS and no barriers are used.
#pragma once

#include "rd_device.h"

namespace rd {

struct FwdArgs {
  const double* in[kMaxFields];
  double* out[kMaxFields];
  KConst c;
};

template <int NS> struct Scheme;
// Euler: z' = z + dt k1.
template <> struct Scheme<1> {
  __device__ static double next_coef(const KConst&, int) { return 0.0; }
};
// Heun: Y2 = z + dt k1, z' = z + (dt/2)(k1 + k2).
template <> struct Scheme<2> {
  __device__ static double next_coef(const KConst& c, int) { return c.dt; }
};
// RK4: Y2 = z + (dt/2) k1, Y3 = z + (dt/2) k2, Y4 = z + dt k3,
// z' = z + (dt/6)(((k1 + 2 k2) + 2 k3) + k4).
template <> struct Scheme<4> {
  __device__ static double next_coef(const KConst& c, int s) { return s < 3 ? c.h2 : c.dt; }
};

template <int MODEL, int STENCIL, int NS>
__global__ __launch_bounds__(256) void fwd_sweep_kernel(FwdArgs a) {
  constexpr int NV = ModelTraits<MODEL>::NV;
  constexpr int TX = kWave - 2 * NS;
  constexpr int ZR = (NS + 1 > 3) ? NS + 1 : 3;
  const KConst& c = a.c;

  const int lane = threadIdx.x & (kWave - 1);
  const int wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (wid >= c.nsx * c.nby) return;  // whole waves only: no barrier follows
  const int sx = wid % c.nsx;
  const int by = wid / c.nsx;
  const int gx = sx * TX - NS + lane;
  const int cx = min(max(gx, 0), c.nx - 1);
  const bool out_col = lane >= NS && lane < NS + TX && gx < c.nx;
  const Column col = make_column(gx, c, STENCIL == RD_LAP9_ANISO);

  const int yA = by * c.ty;
  const int yB = min(yA + c.ty, c.ny);
  const int r_first = max(yA - NS, 0);
  const int r_last = yB - 1 + NS;
  const int load_end = min(yB + NS, c.ny);
  const size_t nx = (size_t)c.nx;

  double zr[ZR][NV];          // zr[a] = z_n at row r - a
  double acc[NS][NV];         // acc[s-1] = running stage sum of row r - s
  double yu[NS + 1][3];       // stage-s input u at rows r-s+1, r-s, r-s-1
  double yg[NS + 1][NV];      // stage-s input gates at row r - s
  double ygn[NS + 1][NV];     // ... produced this iteration for row r-s+1
#pragma unroll
  for (int k = 0; k < ZR; ++k)
#pragma unroll
    for (int f = 0; f < NV; ++f) zr[k][f] = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k)
#pragma unroll
    for (int f = 0; f < NV; ++f) acc[k][f] = 0.0;
#pragma unroll
  for (int s = 0; s <= NS; ++s) {
    yu[s][0] = yu[s][1] = yu[s][2] = 0.0;
#pragma unroll
    for (int f = 0; f < NV; ++f) yg[s][f] = ygn[s][f] = 0.0;
  }

  for (int r = r_first; r <= r_last; ++r) {
    // Advance the register rings by one row.
#pragma unroll
    for (int k = ZR - 1; k > 0; --k)
#pragma unroll
      for (int f = 0; f < NV; ++f) zr[k][f] = zr[k - 1][f];
#pragma unroll
    for (int k = NS - 1; k > 0; --k)
#pragma unroll
      for (int f = 0; f < NV; ++f) acc[k][f] = acc[k - 1][f];
#pragma unroll
    for (int s = 2; s <= NS; ++s) {
      yu[s][2] = yu[s][1];
      yu[s][1] = yu[s][0];
#pragma unroll
      for (int f = 0; f < NV; ++f) yg[s][f] = ygn[s][f];
    }
    if (r < load_end) {
      const size_t o = (size_t)r * nx + cx;
#pragma unroll
      for (int f = 0; f < NV; ++f) zr[0][f] = a.in[f][o];
    }

#pragma unroll
    for (int s = 1; s <= NS; ++s) {
      const int rho = r - s;
      const int lo = max(yA - (NS - s), 0);
      const int hi = min(yB + (NS - s), c.ny);
      if (rho < lo || rho >= hi) continue;  // wave-uniform

      double y[NV], up, dn;
      if (s == 1) {
#pragma unroll
        for (int f = 0; f < NV; ++f) y[f] = zr[1][f];
        up = zr[2][0];
        dn = zr[0][0];
      } else {
        y[0] = yu[s][1];
#pragma unroll
        for (int f = 1; f < NV; ++f) y[f] = yg[s][f];
        up = yu[s][2];
        dn = yu[s][0];
      }
      if (rho == 0) up = y[0];
      if (rho == c.ny - 1) dn = y[0];

      const double lap = diffusion<STENCIL>(up, y[0], dn, col, rho, c);
      double k[NV];
      Reaction<MODEL>::rates(c, y, k);
      k[0] = lap + k[0];

      if (NS == 1) {
        if (out_col && rho >= yA && rho < yB) {
          const size_t o = (size_t)rho * nx + gx;
#pragma unroll
          for (int f = 0; f < NV; ++f) a.out[f][o] = zr[1][f] + c.dt * k[f];
        }
        continue;
      }
      // stage sum: k1, then + 2 k_s (RK4 middle stages) or + k_s
#pragma unroll
      for (int f = 0; f < NV; ++f) {
        if (s == 1) acc[0][f] = k[f];
        else if (NS == 4 && s < 4) acc[s - 1][f] = acc[s - 1][f] + 2.0 * k[f];
        else acc[s - 1][f] = acc[s - 1][f] + k[f];
      }
      if (s < NS) {
        const double cs = Scheme<NS>::next_coef(c, s);
        yu[s + 1][0] = zr[s][0] + cs * k[0];
#pragma unroll
        for (int f = 1; f < NV; ++f) ygn[s + 1][f] = zr[s][f] + cs * k[f];
      } else if (out_col && rho >= yA && rho < yB) {
        const double bw = NS == 4 ? c.h6 : c.h2;
        const size_t o = (size_t)rho * nx + gx;
#pragma unroll
        for (int f = 0; f < NV; ++f) a.out[f][o] = zr[s][f] + bw * acc[s - 1][f];
      }
    }
  }
}

template <int MODEL, int STENCIL, int NS>
hipError_t launch_fwd_sweep(const FwdArgs& a, hipStream_t stream) {
  const int waves = a.c.nsx * a.c.nby;
  const int blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((fwd_sweep_kernel<MODEL, STENCIL, NS>), dim3(blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

// Dispatch over stencil and scheme for one model (defined in rd_fwd_<model>.hip).
template <int MODEL>
hipError_t launch_fwd_model(int stencil, int scheme, const FwdArgs& a, hipStream_t stream) {
  switch (stencil) {
    case RD_LAP5:
      if (scheme == RD_SCHEME_EULER) return launch_fwd_sweep<MODEL, RD_LAP5, 1>(a, stream);
      if (scheme == RD_SCHEME_HEUN) return launch_fwd_sweep<MODEL, RD_LAP5, 2>(a, stream);
      if (scheme == RD_SCHEME_RK4) return launch_fwd_sweep<MODEL, RD_LAP5, 4>(a, stream);
      break;
    case RD_LAP9:
      if (scheme == RD_SCHEME_EULER) return launch_fwd_sweep<MODEL, RD_LAP9, 1>(a, stream);
      if (scheme == RD_SCHEME_HEUN) return launch_fwd_sweep<MODEL, RD_LAP9, 2>(a, stream);
      if (scheme == RD_SCHEME_RK4) return launch_fwd_sweep<MODEL, RD_LAP9, 4>(a, stream);
      break;
    case RD_LAP9_ANISO:
      if (scheme == RD_SCHEME_EULER) return launch_fwd_sweep<MODEL, RD_LAP9_ANISO, 1>(a, stream);
      if (scheme == RD_SCHEME_HEUN) return launch_fwd_sweep<MODEL, RD_LAP9_ANISO, 2>(a, stream);
      if (scheme == RD_SCHEME_RK4) return launch_fwd_sweep<MODEL, RD_LAP9_ANISO, 4>(a, stream);
      break;
  }
  return hipErrorInvalidValue;
}

// Columns each wave produces for a scheme of `ns` stages.
inline int strip_width(int ns) { return kWave - 2 * ns; }

hipError_t launch_fwd_diffusion(int stencil, int scheme, const FwdArgs& a, hipStream_t stream);
hipError_t launch_fwd_barkley(int stencil, int scheme, const FwdArgs& a, hipStream_t stream);
hipError_t launch_fwd_fk(int stencil, int scheme, const FwdArgs& a, hipStream_t stream);
hipError_t launch_fwd_bocf(int stencil, int scheme, const FwdArgs& a, hipStream_t stream);

}  // namespace rd
