// rd_sweep.h -- fused explicit step: every stage of one Euler / Heun / RK4 step
// (stencil, reaction and Euler-like update, Sect. 4) in a single kernel, for
// the state alone or for the state and a tangent in lockstep.
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
//
// Tangent mode (TAN).  Rows carry 2 NV values: the state and its tangent.
// The stencil is applied to u and to du (it is linear), the reaction is
// evaluated on dual numbers (value and derivative along the tangent), and the
// stage combinations, being linear, act on both halves alike.  The state half
// is bit-identical to the plain step.
#pragma once

#include <type_traits>

#include "rd_device.h"

namespace rd {

constexpr int kMaxPacked = 2 * kMaxFields;

// What a sweep launch produces.
enum SweepMode {
  kModeStep = 0,     // z_{n+1} from z_n
  kModeTangent = 1,  // (z_{n+1}, dz_{n+1}) from (z_n, dz_n)
  kModeStages = 2    // the stage inputs Y_2 .. Y_NS of the step from z_n
};

struct SweepArgs {
  const double* in[kMaxPacked];  // state fields, then tangent fields
  double* out[kMaxPacked];       // step / tangent modes
  double* ys[3][kMaxFields];     // stages mode: Y_{s+1} fields, s = 1 .. NS-1
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

// Waves per SIMD each kernel's register budget is sized for (the largest
// count that still needs no scratch spills once the four stages of a steady
// RK4 iteration are interleaved).
template <int MODEL, int STENCIL, int NS, int MODE> struct SweepOccupancy {
  static constexpr bool heavy = MODEL == RD_MODEL_BOCF && STENCIL == RD_LAP9_ANISO;
  static constexpr int value = MODE == kModeTangent ? (NS == 4 || (NS == 2 && MODEL == RD_MODEL_BOCF) ? 1 : 2)
                               : NS == 4            ? (heavy ? 1 : 2)
                               : NS == 2 && heavy   ? 2
                                                    : 3;
};

// f(std::integral_constant<int, 0>{}), ..., f(std::integral_constant<int, N - 1>{}).
template <int N, int I = 0, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<N, I + 1>(f);
  }
}

// Rows of the state loaded ahead of use (deeper where the per-row arithmetic
// is short and registers are plentiful).
template <int MODEL, int NS, int MODE> struct SweepPrefetch {
  static constexpr int NF = (MODE == kModeTangent ? 2 : 1) * ModelTraits<MODEL>::NV;
  static constexpr int value = NF <= 2 ? 4 : MODE == kModeTangent ? 1 : 2;
};

// One wavefront's share of a sweep: strip wid / nby, band wid % nby of the
// grid described by c, reading `in` and writing `out` (or the stage inputs
// `ys`).  Shared by the single-grid and the batched kernels.
template <int MODEL, int STENCIL, int NS, int MODE, bool EDGE>
__device__ __forceinline__ void sweep_wave_impl(const double* const* in, double* const* out,
                                                double* const (*ys)[kMaxFields], const KConst& c,
                                                int wid) {
  constexpr bool TAN = MODE == kModeTangent;
  constexpr bool STAGES = MODE == kModeStages;
  constexpr int NV = ModelTraits<MODEL>::NV;
  constexpr int NF = TAN ? 2 * NV : NV;  // values per cell carried
  constexpr int ND = TAN ? 2 : 1;        // diffusive components: u (and du)
  constexpr int TX = kWave - 2 * NS;
  constexpr int ZR = (NS + 1 > 3) ? NS + 1 : 3;
  auto comp = [](int d) { return d == 0 ? 0 : NV; };  // index of diffusive component d
  auto diffusive = [](int f) { return f == 0 || (TAN && f == NV); };

  const int lane = threadIdx.x & (kWave - 1);
  const int sx = wid / c.nby;  // bands of one strip are consecutive
  const int by = wid % c.nby;
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

  double zr[ZR][NF];          // zr[a] = z_n at row r - a
  double acc[NS][NF];         // acc[s-1] = running stage sum of row r - s
  double yu[NS + 1][3][ND];   // stage-s input u (du) at rows r-s+1, r-s, r-s-1
  double yg[NS + 1][NF];      // stage-s input, other components, row r - s
  double ygn[NS + 1][NF];     // ... produced this iteration for row r-s+1
#pragma unroll
  for (int k = 0; k < ZR; ++k)
#pragma unroll
    for (int f = 0; f < NF; ++f) zr[k][f] = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k)
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[k][f] = 0.0;
#pragma unroll
  for (int s = 0; s <= NS; ++s) {
#pragma unroll
    for (int d = 0; d < ND; ++d) yu[s][0][d] = yu[s][1][d] = yu[s][2][d] = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) yg[s][f] = ygn[s][f] = 0.0;
  }

  // Rows are prefetched PF iterations ahead, so that PF iterations of
  // arithmetic cover the load latency: pre[p] holds row r + p when iteration
  // r starts.  Loads past the band's last input row re-read that row (in
  // bounds, never used), which keeps the steady iterations free of branches.
  constexpr int PF = SweepPrefetch<MODEL, NS, MODE>::value;
  double pre[PF][NF];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    const int row = min(r_first + p, load_end - 1);
#pragma unroll
    for (int f = 0; f < NF; ++f) pre[p][f] = 0.0;
    if (row >= 0) {
      const size_t o = (size_t)row * nx + cx;
#pragma unroll
      for (int f = 0; f < NF; ++f) pre[p][f] = in[f][o];
    }
  }

  // One iteration: take row r, run stage s on row r - s.  STEADY marks
  // iterations in which every stage is active and the rows involved are
  // interior (no y-mirror): its body is free of branches, so the independent
  // reactions of the stages can be interleaved.  SLOT < 0: the prefetch ring
  // shifts by one row (pre[0] is row r); SLOT = q: the loop is unrolled by PF
  // and slot q holds row r, so no prefetched register is read before its
  // turn (a shift would wait for the youngest load).
  auto iter = [&](int r, auto steady_tag, auto slot_tag) __attribute__((always_inline)) {
    constexpr bool STEADY = decltype(steady_tag)::value;
    constexpr int SLOT = decltype(slot_tag)::value;
    // Advance the register rings by one row.
#pragma unroll
    for (int k = ZR - 1; k > 0; --k)
#pragma unroll
      for (int f = 0; f < NF; ++f) zr[k][f] = zr[k - 1][f];
#pragma unroll
    for (int k = NS - 1; k > 0; --k)
#pragma unroll
      for (int f = 0; f < NF; ++f) acc[k][f] = acc[k - 1][f];
#pragma unroll
    for (int s = 2; s <= NS; ++s) {
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        yu[s][2][d] = yu[s][1][d];
        yu[s][1][d] = yu[s][0][d];
      }
#pragma unroll
      for (int f = 0; f < NF; ++f)
        if (!diffusive(f)) yg[s][f] = ygn[s][f];
    }
    if (STEADY || r < load_end) {
      constexpr int q = SLOT < 0 ? 0 : SLOT;
#pragma unroll
      for (int f = 0; f < NF; ++f) zr[0][f] = pre[q][f];
      if constexpr (SLOT < 0) {
#pragma unroll
        for (int p = 0; p + 1 < PF; ++p)
#pragma unroll
          for (int f = 0; f < NF; ++f) pre[p][f] = pre[p + 1][f];
      }
      const size_t o = (size_t)min(r + PF, load_end - 1) * nx + cx;
#pragma unroll
      for (int f = 0; f < NF; ++f) pre[SLOT < 0 ? PF - 1 : q][f] = in[f][o];
    }

#pragma unroll
    for (int s = 1; s <= NS; ++s) {
      if (STAGES && s == NS) continue;  // k_NS is not a stage input
      const int rho = r - s;
      if (!STEADY) {
        const int lo = max(yA - (NS - s), 0);
        const int hi = min(yB + (NS - s), c.ny);
        if (rho < lo || rho >= hi) continue;  // wave-uniform
      }

      double y[NF], up[ND], dn[ND];
      if (s == 1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) y[f] = zr[1][f];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          up[d] = zr[2][comp(d)];
          dn[d] = zr[0][comp(d)];
        }
      } else {
#pragma unroll
        for (int f = 0; f < NF; ++f)
          if (!diffusive(f)) y[f] = yg[s][f];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          y[comp(d)] = yu[s][1][d];
          up[d] = yu[s][2][d];
          dn[d] = yu[s][0][d];
        }
      }
      if (!STEADY) {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          if (rho == 0) up[d] = y[comp(d)];
          if (rho == c.ny - 1) dn[d] = y[comp(d)];
        }
      }

      double lap[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d)
        lap[d] = diffusion<STENCIL, EDGE, !STEADY>(up[d], y[comp(d)], dn[d], col, rho, c);
      double k[NF];
      eval_rates<MODEL, TAN>(c, y, k);
#pragma unroll
      for (int d = 0; d < ND; ++d) k[comp(d)] = lap[d] + k[comp(d)];

      // the last stage's row lies inside the band in every steady iteration
      const bool last_core = out_col && (STEADY || (rho >= yA && rho < yB));
      if (NS == 1) {
        if (!STAGES && last_core) {
          const size_t o = (size_t)rho * nx + gx;
#pragma unroll
          for (int f = 0; f < NF; ++f) out[f][o] = zr[1][f] + c.dt * k[f];
        }
        continue;
      }
      // stage sum: k1, then + 2 k_s (RK4 middle stages) or + k_s
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        if (s == 1) acc[0][f] = k[f];
        else if (NS == 4 && s < 4) acc[s - 1][f] = acc[s - 1][f] + 2.0 * k[f];
        else acc[s - 1][f] = acc[s - 1][f] + k[f];
      }
      if (s < NS) {
        const double cs = Scheme<NS>::next_coef(c, s);
#pragma unroll
        for (int f = 0; f < NF; ++f)
          if (!diffusive(f)) ygn[s + 1][f] = zr[s][f] + cs * k[f];
#pragma unroll
        for (int d = 0; d < ND; ++d) yu[s + 1][0][d] = zr[s][comp(d)] + cs * k[comp(d)];
        if (STAGES && out_col && rho >= yA && rho < yB) {
          const size_t o = (size_t)rho * nx + gx;
          ys[s - 1][0][o] = yu[s + 1][0][0];
#pragma unroll
          for (int f = 1; f < NV; ++f) ys[s - 1][f][o] = ygn[s + 1][f];
        }
      } else if (!STAGES && last_core) {
        const double bw = NS == 4 ? c.h6 : c.h2;
        const size_t o = (size_t)rho * nx + gx;
#pragma unroll
        for (int f = 0; f < NF; ++f) out[f][o] = zr[s][f] + bw * acc[s - 1][f];
      }
    }
  };

  // Steady iterations: r >= yA + NS (every stage's row is at or past its
  // band start), r >= NS + 1 (no stage on row 0), r < min(yB + NS, ny) (row r
  // is an input row, so no stage runs on row ny - 1 or past its band end).
  // Ramp-up and ramp-down iterations shift the prefetch ring; the steady run
  // between them goes PF rows at a time with fixed slots (its rows r + q sit
  // in slot q because the ring is in order when the run starts and ends).
  using Shift = std::integral_constant<int, -1>;
  const int ss_lo = min(max(yA + NS, NS + 1), r_last + 1);
  const int ss_hi = max(load_end, ss_lo);
  const int ss_end = ss_lo + (ss_hi - ss_lo) / PF * PF;
  int r = r_first;
  for (; r < ss_lo; ++r) iter(r, std::false_type{}, Shift{});
  for (; r < ss_end; r += PF) {
    static_for<PF>([&](auto q) { iter(r + q, std::true_type{}, q); });
  }
  for (; r <= r_last; ++r) {
    if (r < ss_hi)
      iter(r, std::true_type{}, Shift{});
    else
      iter(r, std::false_type{}, Shift{});
  }
}

// Strips that touch the grid's x-edges apply the mirror; interior strips skip it.
template <int MODEL, int STENCIL, int NS, int MODE>
__device__ __forceinline__ void sweep_wave(const double* const* in, double* const* out,
                                           double* const (*ys)[kMaxFields], const KConst& c,
                                           int wid) {
  const int x0 = (wid / c.nby) * (kWave - 2 * NS) - NS;
  if (strip_touches_edge(x0, c))
    sweep_wave_impl<MODEL, STENCIL, NS, MODE, true>(in, out, ys, c, wid);
  else
    sweep_wave_impl<MODEL, STENCIL, NS, MODE, false>(in, out, ys, c, wid);
}

template <int MODEL, int STENCIL, int NS, int MODE>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(SweepOccupancy<MODEL, STENCIL, NS, MODE>::value)))
void sweep_kernel(SweepArgs a) {
  const int blk = xcd_order((int)blockIdx.x, (int)gridDim.x);
  const int wid = __builtin_amdgcn_readfirstlane(blk * (int)(blockDim.x / kWave) + (int)(threadIdx.x / kWave));
  if (wid >= a.c.nsx * a.c.nby) return;  // whole waves only: no barrier follows
  sweep_wave<MODEL, STENCIL, NS, MODE>(a.in, a.out, a.ys, a.c, wid);
}

template <int MODEL, int STENCIL, int NS, int MODE>
hipError_t launch_sweep(const SweepArgs& a, hipStream_t stream) {
  if (MODE == kModeStages && NS == 1) return hipSuccess;  // Euler has no inner stage
  const int waves = a.c.nsx * a.c.nby;
  const int blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((sweep_kernel<MODEL, STENCIL, NS, MODE>), dim3(blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

// Dispatch over stencil and scheme for one model and mode.
template <int MODEL, int MODE>
hipError_t launch_sweep_model(int stencil, int scheme, const SweepArgs& a, hipStream_t s) {
  switch (stencil) {
    case RD_LAP5:
      if (scheme == RD_SCHEME_EULER) return launch_sweep<MODEL, RD_LAP5, 1, MODE>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_sweep<MODEL, RD_LAP5, 2, MODE>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_sweep<MODEL, RD_LAP5, 4, MODE>(a, s);
      break;
    case RD_LAP9:
      if (scheme == RD_SCHEME_EULER) return launch_sweep<MODEL, RD_LAP9, 1, MODE>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_sweep<MODEL, RD_LAP9, 2, MODE>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_sweep<MODEL, RD_LAP9, 4, MODE>(a, s);
      break;
    case RD_LAP9_ANISO:
      if (scheme == RD_SCHEME_EULER) return launch_sweep<MODEL, RD_LAP9_ANISO, 1, MODE>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_sweep<MODEL, RD_LAP9_ANISO, 2, MODE>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_sweep<MODEL, RD_LAP9_ANISO, 4, MODE>(a, s);
      break;
  }
  return hipErrorInvalidValue;
}

// Columns each wave produces for a scheme of `ns` stages.
inline int strip_width(int ns) { return kWave - 2 * ns; }

// One fused step of the state (fwd), of state and tangent (tan), or the
// stage inputs of a step (stg), defined per model in rd_sweep_<kind>_<model>.hip.
#define RD_DECLARE_SWEEP(kind, model) \
  hipError_t launch_sweep_##kind##_##model(int stencil, int scheme, const SweepArgs& a, hipStream_t s);
RD_DECLARE_SWEEP(fwd, diffusion)
RD_DECLARE_SWEEP(fwd, barkley)
RD_DECLARE_SWEEP(fwd, fk)
RD_DECLARE_SWEEP(fwd, bocf)
RD_DECLARE_SWEEP(tan, diffusion)
RD_DECLARE_SWEEP(tan, barkley)
RD_DECLARE_SWEEP(tan, fk)
RD_DECLARE_SWEEP(tan, bocf)
RD_DECLARE_SWEEP(stg, diffusion)
RD_DECLARE_SWEEP(stg, barkley)
RD_DECLARE_SWEEP(stg, fk)
RD_DECLARE_SWEEP(stg, bocf)
#undef RD_DECLARE_SWEEP
#define RD_DECLARE_PIPE(kind, model) \
  hipError_t launch_pipe_##kind##_##model(int stencil, int scheme, const SweepArgs& a, hipStream_t s);
RD_DECLARE_PIPE(fwd, diffusion)
RD_DECLARE_PIPE(fwd, barkley)
RD_DECLARE_PIPE(fwd, fk)
RD_DECLARE_PIPE(fwd, bocf)
RD_DECLARE_PIPE(tan, diffusion)
RD_DECLARE_PIPE(tan, barkley)
RD_DECLARE_PIPE(tan, fk)
RD_DECLARE_PIPE(tan, bocf)
RD_DECLARE_PIPE(stg, diffusion)
RD_DECLARE_PIPE(stg, barkley)
RD_DECLARE_PIPE(stg, fk)
RD_DECLARE_PIPE(stg, bocf)
#undef RD_DECLARE_PIPE

// Kernel variants of the fused step (identical results): one wave carrying
// every stage (rd_sweep.h) or one wave per stage (rd_pipe.h).
enum StepVariant { kVariantSweep = 0, kVariantPipe = 1 };

// Dispatch over models.
hipError_t launch_sweep_mode(int mode, int model, int stencil, int scheme, const SweepArgs& a,
                             hipStream_t s);

}  // namespace rd
