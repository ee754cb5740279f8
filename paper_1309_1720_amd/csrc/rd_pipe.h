// rd_pipe.h -- fused explicit step, stage-pipelined across the waves of a
// workgroup.
//
// A workgroup owns the same 64-column strip and row band as one wave of the
// sweep kernel (rd_sweep.h), but it has NS waves and wave s runs only stage s
// of the Euler / Heun / RK4 step.  All waves step through the band together,
// one row per iteration, wave s two rows behind wave s - 1:
//
//   iteration t:  wave s processes row base + t - 2 (s - 1)
//
// so every value a wave reads was written by another wave in an earlier
// iteration, and one workgroup barrier per iteration orders them.  Between
// stages the data travels through small LDS row rings:
//   U[s]  the diffusive component(s) of the stage input Y_s, 4 rows (the
//         stencil reads rows rho - 1 .. rho + 1 while row rho + 2 is written);
//   G[s]  the other components of Y_s, 3 rows;
//   A[s]  the running stage sum handed to stage s, 3 rows.
// Wave 1 fills U[1] with the state two rows ahead of its own row; each wave
// loads z_n of its own row (prefetched one iteration ahead) for the update
// Y_{s+1} = z_n + c_s dt k_s.  Neighbouring columns are read from the LDS
// rows, the x-mirror by choosing the index and the y-mirror by clamping the
// row, so the stencil needs no selects.  Compared with one wave carrying all
// stages, each wave holds a quarter of the state in registers (more waves per
// SIMD) and bands can be taller for the same number of waves (less halo).
//
// The arithmetic is that of the sweep kernel, in the same order: both
// produce identical bits.
#pragma once

#include "rd_sweep.h"

namespace rd {

constexpr int kPad = kWave + 2;  // LDS row: 64 lanes and a pad column on each side

template <int MODEL, int NS, int MODE> struct PipeShape {
  static constexpr int NV = ModelTraits<MODEL>::NV;
  static constexpr int NDF = ModelTraits<MODEL>::NDIFF;
  static constexpr int NF = (MODE == kModeTangent ? 2 : 1) * NV;
  static constexpr int ND = (MODE == kModeTangent ? 2 : 1) * NDF;
  static constexpr int NG = NF - ND;
  static constexpr int NI = NS > 1 ? NS - 1 : 1;  // stages fed through G and A
  static constexpr int U_doubles = NS * 4 * ND * kPad;
  static constexpr int G_doubles = NI * 3 * (NG > 0 ? NG : 1) * kWave;
  static constexpr int A_doubles = NI * 3 * NF * kWave;
  static constexpr int total = U_doubles + G_doubles + A_doubles;
};

template <int MODEL, int STENCIL, int NS, int MODE, bool EDGE, int HK>
__device__ __forceinline__ void pipe_block_impl(const double* const* in, double* const* out,
                                                double* const (*ys)[kMaxFields], const KConst& c,
                                                int blk, double* lds) {
  using Sh = PipeShape<MODEL, NS, MODE>;
  constexpr int NV = Sh::NV, NDF = Sh::NDF, NF = Sh::NF, ND = Sh::ND, NG = Sh::NG;
  constexpr bool TAN = MODE == kModeTangent;
  constexpr bool STAGES = MODE == kModeStages;
  constexpr int TX = kWave - 2 * NS;
  // packed index of diffusive component d, whether packed value f diffuses,
  // and the index of a non-diffusive value among the non-diffusive ones
  auto comp = [](int d) { return d < NDF ? d : NV + (d - NDF); };
  auto diffusive = [](int f) { return f < NDF || (TAN && f >= NV && f - NV < NDF); };
  auto gidx = [](int f) { return f < NV ? f - NDF : (NV - NDF) + (f - NV - NDF); };

  const int lane = threadIdx.x & (kWave - 1);
  const int s = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)) + 1;  // this wave's stage
  const int sx = blk / c.nby;  // bands of one strip are consecutive
  const int by = blk % c.nby;
  const int gx = sx * TX - NS + lane;
  const int cx = min(max(gx, 0), c.nx - 1);
  const bool out_col = lane >= NS && lane < NS + TX && gx < c.nx;
  const Column col = make_column(gx, c, STENCIL == RD_LAP9_ANISO);
  const int il = lane + 1;
  const int iw = (EDGE && col.west) ? il : il - 1;
  const int ie = (EDGE && col.east) ? il : il + 1;
  const size_t nx = (size_t)c.nx;

  const int yA = by * c.ty;
  const int yB = min(yA + c.ty, c.ny);
  const int base = max(yA - (NS - 1), 0);                 // first row of stage 1
  const int last = min(yB, c.ny) - 1;                     // last row of stage NS
  const int iters = last - base + 2 * (NS - 1) + 1;
  const int my_lo = max(yA - (NS - s), 0);
  const int my_hi = min(yB + (NS - s), c.ny);
  const int load_end = min(yB + NS, c.ny);               // stage-1 input rows end here

  double* const U0 = lds;
  double* const G0 = lds + Sh::U_doubles;
  double* const A0 = lds + Sh::U_doubles + Sh::G_doubles;
  auto urow = [&](int st, int row, int d) { return U0 + (((st - 1) * 4 + (row & 3)) * ND + d) * kPad; };
  auto grow = [&](int st, int row) { return G0 + ((st - 2) * 3 + row % 3) * (NG > 0 ? NG : 1) * kWave; };
  auto arow = [&](int st, int row) { return A0 + ((st - 2) * 3 + row % 3) * NF * kWave; };

  // Wave 1 seeds U[1] with the first three rows its stencil reads.
  if (s == 1) {
    for (int row = base - 1; row <= base + 1; ++row)
      if (row >= 0 && row < c.ny)
#pragma unroll
        for (int d = 0; d < ND; ++d) urow(1, row, d)[il] = in[comp(d)][(size_t)row * nx + cx];
  }
  double pre[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) pre[f] = 0.0;
  if (my_lo < my_hi) {
#pragma unroll
    for (int f = 0; f < NF; ++f) pre[f] = in[f][(size_t)my_lo * nx + cx];
  }
  __syncthreads();

  for (int t = 0; t < iters; ++t) {
    const int rho = base + t - 2 * (s - 1);
    // wave-uniform; in stages mode the last stage has nothing to produce
    const bool active = rho >= my_lo && rho < my_hi && !(STAGES && s == NS);
    // wave 1: the state row two ahead, stored into U[1] after this iteration's reads
    const int wrow = base + t + 2;
    const bool feed = s == 1 && wrow < load_end;
    double unext[ND];
    if (feed) {
#pragma unroll
      for (int d = 0; d < ND; ++d) unext[d] = in[comp(d)][(size_t)wrow * nx + cx];
    }
    if (active) {
      double zc[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) zc[f] = pre[f];
      if (rho + 1 < my_hi) {
        const size_t o = (size_t)(rho + 1) * nx + cx;
#pragma unroll
        for (int f = 0; f < NF; ++f) pre[f] = in[f][o];
      }
      // stage input Y_s at row rho
      double y[NF];
      const int ru = rho > 0 ? rho - 1 : 0;
      const int rd = rho < c.ny - 1 ? rho + 1 : rho;
      if (s == 1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) y[f] = zc[f];
      } else {
        const double* g = grow(s, rho);
#pragma unroll
        for (int f = 0; f < NF; ++f)
          if (!diffusive(f)) y[f] = g[gidx(f) * kWave + lane];
#pragma unroll
        for (int d = 0; d < ND; ++d) y[comp(d)] = urow(s, rho, d)[il];
      }
      double lap[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d)
        lap[d] = diffusion_rows<STENCIL, EDGE>(urow(s, ru, d), urow(s, rho, d), urow(s, rd, d), il, iw, ie,
                                               col, rho, c, c.dcoef[d % NDF]);
      double k[NF];
      eval_rates<MODEL, TAN, HK>(c, y, k);
#pragma unroll
      for (int d = 0; d < ND; ++d) k[comp(d)] = lap[d] + k[comp(d)];

      const bool core = out_col && rho >= yA && rho < yB;
      if (NS == 1) {
        if (!STAGES && core) {
          const size_t o = (size_t)rho * nx + gx;
#pragma unroll
          for (int f = 0; f < NF; ++f) out[f][o] = zc[f] + c.dt * k[f];
        }
      } else {
        double acc[NF];
        if (s == 1) {
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[f] = k[f];
        } else {
          const double* ap = arow(s, rho);
          const bool twice = NS == 4 && s < 4;  // RK4: k1 + 2 k2 + 2 k3 + k4
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[f] = ap[f * kWave + lane] + (twice ? 2.0 * k[f] : k[f]);
        }
        if (s < NS) {
          const double cs = Scheme<NS>::next_coef(c, s);
          double yn[NF];
#pragma unroll
          for (int f = 0; f < NF; ++f) yn[f] = zc[f] + cs * k[f];
#pragma unroll
          for (int d = 0; d < ND; ++d) urow(s + 1, rho, d)[il] = yn[comp(d)];
          double* g = grow(s + 1, rho);
          double* ap = arow(s + 1, rho);
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            if (!diffusive(f)) g[gidx(f) * kWave + lane] = yn[f];
            ap[f * kWave + lane] = acc[f];
          }
          if (STAGES && core) {
            const size_t o = (size_t)rho * nx + gx;
#pragma unroll
            for (int f = 0; f < NV; ++f) ys[s - 1][f][o] = yn[f];
          }
        } else if (!STAGES && core) {
          const double bw = NS == 4 ? c.h6 : c.h2;
          const size_t o = (size_t)rho * nx + gx;
#pragma unroll
          for (int f = 0; f < NF; ++f) out[f][o] = zc[f] + bw * acc[f];
        }
      }
    }
    if (feed) {
#pragma unroll
      for (int d = 0; d < ND; ++d) urow(1, wrow, d)[il] = unext[d];
    }
    __syncthreads();
  }
}

template <int MODEL, int STENCIL, int NS, int MODE, int HK>
__device__ __forceinline__ void pipe_block(const double* const* in, double* const* out,
                                           double* const (*ys)[kMaxFields], const KConst& c, int blk,
                                           double* lds) {
  const int x0 = (blk / c.nby) * (kWave - 2 * NS) - NS;
  if (strip_touches_edge(x0, c))
    pipe_block_impl<MODEL, STENCIL, NS, MODE, true, HK>(in, out, ys, c, blk, lds);
  else
    pipe_block_impl<MODEL, STENCIL, NS, MODE, false, HK>(in, out, ys, c, blk, lds);
}

template <int MODEL, int STENCIL, int NS, int MODE, int HK>
__global__ __launch_bounds__(kWave * NS) void pipe_kernel(SweepArgs a) {
  __shared__ double lds[PipeShape<MODEL, NS, MODE>::total];
  pipe_block<MODEL, STENCIL, NS, MODE, HK>(a.in, a.out, a.ys, a.c, xcd_order((int)blockIdx.x, (int)gridDim.x), lds);
}

template <int MODEL, int STENCIL, int NS, int MODE, int HK>
hipError_t launch_pipe(const SweepArgs& a, hipStream_t stream) {
  if (MODE == kModeStages && NS == 1) return hipSuccess;  // Euler has no inner stage
  hipLaunchKernelGGL((pipe_kernel<MODEL, STENCIL, NS, MODE, HK>), dim3(a.c.nsx * a.c.nby), dim3(kWave * NS),
                     0, stream, a);
  return hipGetLastError();
}

template <int MODEL, int MODE, int HK>
hipError_t launch_pipe_model_hk(int stencil, int scheme, const SweepArgs& a, hipStream_t s) {
  switch (stencil) {
    case RD_LAP5:
      if (scheme == RD_SCHEME_EULER) return launch_pipe<MODEL, RD_LAP5, 1, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_pipe<MODEL, RD_LAP5, 2, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_pipe<MODEL, RD_LAP5, 4, MODE, HK>(a, s);
      break;
    case RD_LAP9:
      if (scheme == RD_SCHEME_EULER) return launch_pipe<MODEL, RD_LAP9, 1, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_pipe<MODEL, RD_LAP9, 2, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_pipe<MODEL, RD_LAP9, 4, MODE, HK>(a, s);
      break;
    case RD_LAP9_ANISO:
      if (scheme == RD_SCHEME_EULER) return launch_pipe<MODEL, RD_LAP9_ANISO, 1, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_pipe<MODEL, RD_LAP9_ANISO, 2, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_pipe<MODEL, RD_LAP9_ANISO, 4, MODE, HK>(a, s);
      break;
  }
  return hipErrorInvalidValue;
}

// Models with H_k run the smooth or the sharp evaluation of it (as the sweep
// kernels do, so that both variants give the same bits).
template <int MODEL, int MODE>
hipError_t launch_pipe_model(int stencil, int scheme, const SweepArgs& a, hipStream_t s) {
  if constexpr (ModelTraits<MODEL>::GATED) {
    return a.c.sharp ? launch_pipe_model_hk<MODEL, MODE, kHkSharp>(stencil, scheme, a, s)
                     : launch_pipe_model_hk<MODEL, MODE, kHkSmooth>(stencil, scheme, a, s);
  } else {
    return launch_pipe_model_hk<MODEL, MODE, kHkAny>(stencil, scheme, a, s);
  }
}

}  // namespace rd
