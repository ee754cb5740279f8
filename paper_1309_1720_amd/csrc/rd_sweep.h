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

// Steps one launch may advance (temporal blocking): the state-only sweep of
// the models with cheap reactions chains up to 8 stages, so that a launch
// reads and writes the state once for several steps.  1 elsewhere.
template <int MODEL, int NS, int MODE> struct MultiStep {
  static constexpr int max =
      MODE == kModeStep && (MODEL == RD_MODEL_DIFFUSION || MODEL == RD_MODEL_BARKLEY || MODEL == RD_MODEL_FHN)
          ? 8 / NS
          : 1;
};

// Waves per SIMD each kernel's register budget is sized for (the largest
// count that still needs no scratch spills once the stages of a steady
// iteration are interleaved).
template <int MODEL, int STENCIL, int NS, int MODE, int K = 1> struct SweepOccupancy {
  static constexpr bool heavy = MODEL == RD_MODEL_BOCF && STENCIL == RD_LAP9_ANISO;
  static constexpr int value = K > 1                ? 2
                               : MODE == kModeTangent ? (NS == 4 || (NS == 2 && MODEL == RD_MODEL_BOCF) ? 1 : 2)
                               : NS == 4            ? 2
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

// Waves per workgroup of the sweep kernels (consecutive bands of a strip).
constexpr int kSweepWaves = 4;

// The boundary rule inside a sweep: read from the constants at run time, or
// compiled in (no-flux, periodic).  Compiled in, its tests fold and the
// steady iterations lose their wrap logic and the scalar registers it holds
// (FK 1024^2 23.8 -> 22.7 us); the Bueno-Orovio step measured slower that way
// (148 -> 156-163 us) and reads it at run time.
enum { kBoundaryRuntime = 0, kBoundaryNoFlux = 1, kBoundaryPeriodic = 2 };

// Kernel variants of the fused step (identical results): one wave carrying
// every stage (rd_sweep.h) or one wave per stage (rd_pipe.h).
enum StepVariant { kVariantSweep = 0, kVariantPipe = 1 };

// Rows of the state loaded ahead of use (deeper where the per-row arithmetic
// is short and registers are plentiful).
template <int MODEL, int NS, int MODE> struct SweepPrefetch {
  static constexpr int NF = (MODE == kModeTangent ? 2 : 1) * ModelTraits<MODEL>::NV;
  static constexpr int value = NF <= 2 ? 4 : MODE == kModeTangent ? 1 : 2;
};

// One wavefront's share of a sweep: strip wid / nby, band wid % nby of the
// grid described by c, reading `in` and writing `out` (or the stage inputs
// `ys`), advancing K steps (K > 1 only for the plain step).  GATE selects a
// one-stage gate scheme (1 Rush-Larsen, 2 implicit Euler; NS = 1, gated
// models) instead of explicit Euler.  Shared by the single-grid and the
// batched kernels.
//
// K steps chain K copies of the one-step pipeline: copy k takes row r - k NS
// of z_{n+k} (the row copy k - 1 finished in the same iteration; copy 0 the
// row just loaded) and runs its stage s on row r - k NS - s, so the launch
// needs KS = K NS halo columns and ramp rows.
// FR: ramp-up iterations with compile-time stage activity (below), and the
// steady run unrolled by at least two rows; off, the former loop structure
// (kept where it measured faster: the batched tangent step).
template <int MODEL, int STENCIL, int NS, int MODE, bool EDGE, int K = 1, int GATE = 0, int HK = kHkAny,
          bool FR = true, int PB = kBoundaryRuntime>
__device__ __forceinline__ void sweep_wave_impl(const double* const* in, double* const* out,
                                                double* const (*ys)[kMaxFields], const KConst& c,
                                                int wid) {
  // PB: the boundary rule read from c, or fixed at compile time (its tests
  // then fold); row indices wrap (periodic) or clamp (no-flux)
  const bool PER = PB == kBoundaryRuntime ? c.periodic != 0 : PB == kBoundaryPeriodic;
  auto row_index = [&](int y) { return PER ? wrap_index(y, c.ny) : min(max(y, 0), c.ny - 1); };
  static_assert(K == 1 || MODE == kModeStep, "several steps per launch advance the state only");
  static_assert(GATE == 0 || (NS == 1 && K == 1), "gate schemes have one stage");
  constexpr bool TAN = MODE == kModeTangent;
  constexpr bool STAGES = MODE == kModeStages;
  constexpr int NV = ModelTraits<MODEL>::NV;
  constexpr int NDF = ModelTraits<MODEL>::NDIFF;  // diffusive fields: 0 .. NDF-1
  constexpr int NF = TAN ? 2 * NV : NV;           // values per cell carried
  constexpr int ND = TAN ? 2 * NDF : NDF;         // diffusive components (and their tangents)
  constexpr int KS = K * NS;                      // stages per launch
  constexpr int TX = kWave - 2 * KS;
  constexpr int ZR = (NS + 1 > 3) ? NS + 1 : 3;
  // packed index of diffusive component d, and whether packed value f diffuses
  auto comp = [](int d) { return d < NDF ? d : NV + (d - NDF); };
  auto diffusive = [](int f) { return f < NDF || (TAN && f >= NV && f - NV < NDF); };

  const int lane = threadIdx.x & (kWave - 1);
  const int sx = wid / c.nby;  // bands of one strip are consecutive
  const int by = wid % c.nby;
  const int gx = sx * TX - KS + lane;
  const int cx = PER ? wrap_index(gx, c.nx) : min(max(gx, 0), c.nx - 1);
  const bool out_col = lane >= KS && lane < KS + TX && gx < c.nx;
  const Column col = make_column(gx, c, STENCIL == RD_LAP9_ANISO);

  const int yA = by * c.ty;
  const int yB = min(yA + c.ty, c.ny);
  // periodic grids run the ramps through the wrapped rows
  const int r_first = PER ? yA - KS : max(yA - KS, 0);
  const int r_last = yB - 1 + KS;
  const int load_end = PER ? yB + KS : min(yB + KS, c.ny);
  const size_t nx = (size_t)c.nx;

  // Per step copy k: register rings indexed by rows relative to its input row
  // r - k NS.
  double zr[K][ZR][NF];          // z_{n+k} at row (r - k NS) - a
  double acc[K][NS][NF];         // running stage sum of row (r - k NS) - s
  double yu[K][NS + 1][3][ND];   // stage-s input u (du), rows (r - k NS) - s + 1 .. - s - 1
  double yg[K][NS + 1][NF];      // stage-s input, other components, row (r - k NS) - s
  double ygn[K][NS + 1][NF];     // ... produced this iteration for the row below it
  // anisotropic flux form: the south-face flux each stage computed on the row above
  constexpr bool CARRY = STENCIL == RD_LAP9_ANISO;
  double fyc[K][NS + 1][ND];
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int a = 0; a < ZR; ++a)
#pragma unroll
      for (int f = 0; f < NF; ++f) zr[k][a][f] = 0.0;
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
      for (int f = 0; f < NF; ++f) acc[k][a][f] = 0.0;
#pragma unroll
    for (int s = 0; s <= NS; ++s) {
#pragma unroll
      for (int d = 0; d < ND; ++d) yu[k][s][0][d] = yu[k][s][1][d] = yu[k][s][2][d] = 0.0;
#pragma unroll
      for (int f = 0; f < NF; ++f) yg[k][s][f] = ygn[k][s][f] = 0.0;
#pragma unroll
      for (int d = 0; d < ND; ++d) fyc[k][s][d] = 0.0;
    }
  }

  // Rows are prefetched PF iterations ahead, so that PF iterations of
  // arithmetic cover the load latency: pre[p] holds row r + p when iteration
  // r starts.  Loads past the band's last input row re-read that row (in
  // bounds, never used), which keeps the steady iterations free of branches.
  constexpr int PF = SweepPrefetch<MODEL, NS, MODE>::value;
  double pre[PF][NF];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    const int row = row_index(min(r_first + p, load_end - 1));
#pragma unroll
    for (int f = 0; f < NF; ++f) pre[p][f] = 0.0;
    if (row >= 0) {
      const size_t o = (size_t)row * nx + cx;
#pragma unroll
      for (int f = 0; f < NF; ++f) pre[p][f] = in[f][o];
    }
  }

  // One iteration: take row r; step copy k runs stage s on row r - k NS - s.
  // STEADY marks iterations in which every stage is active and the rows
  // involved are interior (no y-mirror): its body is free of branches, so the
  // independent reactions of the stages can be interleaved.  SLOT < 0: the
  // prefetch ring shifts by one row (pre[0] is row r); SLOT = q: the loop is
  // unrolled by PF and slot q holds row r, so no prefetched register is read
  // before its turn (a shift would wait for the youngest load).
  //
  // PHASE = 1 + i: ramp-up iteration i (row yA - KS + i) of a band away from
  // the y-edges, where which stages run is known at compile time (copy k runs
  // stage s from i = 2 (k NS + s) on).  Such iterations, like the steady
  // ones, test no ranges, apply no y-mirror and store without a row test;
  // PHASE = 0 is the general ramp iteration.
  auto iter = [&](int r, auto steady_tag, auto slot_tag, auto phase_tag) __attribute__((always_inline)) {
    constexpr bool STEADY = decltype(steady_tag)::value;
    constexpr int SLOT = decltype(slot_tag)::value;
    constexpr int PHASE = STEADY ? 0 : decltype(phase_tag)::value;
    constexpr bool UP = PHASE > 0;
    constexpr bool FIXED = STEADY || UP;
    // Advance the register rings by one row.
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int a = ZR - 1; a > 0; --a)
#pragma unroll
        for (int f = 0; f < NF; ++f) zr[k][a][f] = zr[k][a - 1][f];
#pragma unroll
      for (int a = NS - 1; a > 0; --a)
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[k][a][f] = acc[k][a - 1][f];
#pragma unroll
      for (int s = 2; s <= NS; ++s) {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          yu[k][s][2][d] = yu[k][s][1][d];
          yu[k][s][1][d] = yu[k][s][0][d];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f)
          if (!diffusive(f)) yg[k][s][f] = ygn[k][s][f];
      }
    }
    if (FIXED || r < load_end) {
      constexpr int q = SLOT < 0 ? 0 : SLOT;
#pragma unroll
      for (int f = 0; f < NF; ++f) zr[0][0][f] = pre[q][f];
      if constexpr (SLOT < 0) {
#pragma unroll
        for (int p = 0; p + 1 < PF; ++p)
#pragma unroll
          for (int f = 0; f < NF; ++f) pre[p][f] = pre[p + 1][f];
      }
      const size_t o = (size_t)row_index(min(r + PF, load_end - 1)) * nx + cx;
#pragma unroll
      for (int f = 0; f < NF; ++f) pre[SLOT < 0 ? PF - 1 : q][f] = in[f][o];
    }

    double zout[NF];  // row r - (k + 1) NS of z_{n+k+1}, handed to copy k + 1
#pragma unroll
    for (int f = 0; f < NF; ++f) zout[f] = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k > 0) {
        // the row copy k - 1 finished this iteration (read only inside the
        // range that copy produced)
#pragma unroll
        for (int f = 0; f < NF; ++f) zr[k][0][f] = zout[f];
      }
#pragma unroll
      for (int s = 1; s <= NS; ++s) {
        if (STAGES && s == NS) continue;  // k_NS is not a stage input
        const int rho = r - k * NS - s;
        if (UP) {
          if (PHASE - 1 < 2 * (k * NS + s)) continue;  // folded
        } else if (!STEADY) {
          const int lo = PER ? yA - (K - k) * NS + s : max(yA - (K - k) * NS + s, 0);
          const int hi = PER ? yB + (K - k) * NS - s : min(yB + (K - k) * NS - s, c.ny);
          if (rho < lo || rho >= hi) continue;  // wave-uniform
        }

        double y[NF], up[ND], dn[ND];
        if (s == 1) {
#pragma unroll
          for (int f = 0; f < NF; ++f) y[f] = zr[k][1][f];
#pragma unroll
          for (int d = 0; d < ND; ++d) {
            up[d] = zr[k][2][comp(d)];
            dn[d] = zr[k][0][comp(d)];
          }
        } else {
#pragma unroll
          for (int f = 0; f < NF; ++f)
            if (!diffusive(f)) y[f] = yg[k][s][f];
#pragma unroll
          for (int d = 0; d < ND; ++d) {
            y[comp(d)] = yu[k][s][1][d];
            up[d] = yu[k][s][2][d];
            dn[d] = yu[k][s][0][d];
          }
        }
        if (!FIXED) {
#pragma unroll
          for (int d = 0; d < ND; ++d) {
            if (!PER && rho == 0) up[d] = y[comp(d)];
            if (!PER && rho == c.ny - 1) dn[d] = y[comp(d)];
          }
        }

        double lap[ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          if constexpr (CARRY)
            lap[d] = diffusion_flux_rows<EDGE, !FIXED, STEADY>(up[d], y[comp(d)], dn[d], col, rho, c,
                                                               c.dcoef[d % NDF], fyc[k][s][d]);
          else
            lap[d] = diffusion<STENCIL, EDGE, !FIXED>(up[d], y[comp(d)], dn[d], col, rho, c, c.dcoef[d % NDF]);
        }
        double kr[NF];
        eval_rates<MODEL, TAN, HK>(c, y, kr);
#pragma unroll
        for (int d = 0; d < ND; ++d) kr[comp(d)] = lap[d] + kr[comp(d)];

        // the last stage's row lies inside the band in every steady or fixed iteration
        const bool last = k == K - 1;
        const bool last_core = out_col && (FIXED || (rho >= yA && rho < yB));
        if (NS == 1) {
          if (STAGES) continue;
          double zn[NF];
          if constexpr (GATE == 0) {
#pragma unroll
            for (int f = 0; f < NF; ++f) zn[f] = zr[k][1][f] + c.dt * kr[f];
          } else {
            gate_scheme_step<MODEL, TAN, GATE, HK>(c, zr[k][1], kr, zn);
          }
          if (!last) {
#pragma unroll
            for (int f = 0; f < NF; ++f) zout[f] = zn[f];
          } else if (last_core) {
            const size_t o = (size_t)rho * nx + gx;
#pragma unroll
            for (int f = 0; f < NF; ++f) out[f][o] = zn[f];
          }
          continue;
        }
        // stage sum: k1, then + 2 k_s (RK4 middle stages) or + k_s
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          if (s == 1) acc[k][0][f] = kr[f];
          else if (NS == 4 && s < 4) acc[k][s - 1][f] = acc[k][s - 1][f] + 2.0 * kr[f];
          else acc[k][s - 1][f] = acc[k][s - 1][f] + kr[f];
        }
        if (s < NS) {
          const double cs = Scheme<NS>::next_coef(c, s);
#pragma unroll
          for (int f = 0; f < NF; ++f)
            if (!diffusive(f)) ygn[k][s + 1][f] = zr[k][s][f] + cs * kr[f];
#pragma unroll
          for (int d = 0; d < ND; ++d) yu[k][s + 1][0][d] = zr[k][s][comp(d)] + cs * kr[comp(d)];
          if (STAGES && out_col && rho >= yA && rho < yB) {
            const size_t o = (size_t)rho * nx + gx;
#pragma unroll
            for (int f = 0; f < NV; ++f) ys[s - 1][f][o] = f < NDF ? yu[k][s + 1][0][f] : ygn[k][s + 1][f];
          }
        } else if (!STAGES) {
          const double bw = NS == 4 ? c.h6 : c.h2;
          if (!last) {
#pragma unroll
            for (int f = 0; f < NF; ++f) zout[f] = zr[k][s][f] + bw * acc[k][s - 1][f];
          } else if (last_core) {
            const size_t o = (size_t)rho * nx + gx;
#pragma unroll
            for (int f = 0; f < NF; ++f) out[f][o] = zr[k][s][f] + bw * acc[k][s - 1][f];
          }
        }
      }
    }
  };

  // Steady iterations: r >= yA + KS (every stage's row is at or past its
  // range start), r >= KS + 1 (no stage on row 0), r < min(yB + KS, ny) (row r
  // is an input row, so no stage runs on row ny - 1 or past its range end).
  // Ramp-up and ramp-down iterations shift the prefetch ring; the steady run
  // between them goes PF rows at a time with fixed slots (its rows r + q sit
  // in slot q because the ring is in order when the run starts and ends).
  using Shift = std::integral_constant<int, -1>;
  // (one iteration later with the carried face fluxes: every stage must have
  // run on the row above its first steady row)
  constexpr int CL = CARRY ? 1 : 0;
  const int ss_lo = min(PER ? yA + KS + CL : max(yA + KS + CL, KS + 1), r_last + 1);
  const int ss_hi = max(load_end, ss_lo);
  const int ss_end = ss_lo + (ss_hi - ss_lo) / PF * PF;
  using Gen = std::integral_constant<int, 0>;
  int r = r_first;
  if constexpr (!FR) {
    for (; r < ss_lo; ++r) iter(r, std::false_type{}, Shift{}, Gen{});
    for (; r < ss_end; r += PF) {
      static_for<PF>([&](auto q) { iter(r + q, std::true_type{}, q, Gen{}); });
    }
    for (; r <= r_last; ++r) {
      if (r < ss_hi)
        iter(r, std::true_type{}, Shift{}, Gen{});
      else
        iter(r, std::false_type{}, Shift{}, Gen{});
    }
    return;
  }
  // Fixed ramp-up: rows r_first = yA - KS .. ss_lo - 1 lie at least one row
  // inside both y-edges (stage rows yA - KS + s .. yA + KS + CL - 2), and
  // every stage row is before its range end.
  if (!PER && yA >= KS && yA + 2 * KS + 1 < c.ny) {
    static_for<2 * KS + CL>([&](auto i) {
      constexpr int I = decltype(i)::value;
      iter(r_first + I, std::false_type{}, Shift{}, std::integral_constant<int, 1 + I>{});
    });
    r = ss_lo;  // = yA + KS + CL here
  }
  // The steady run goes SU rows at a time: PF (slot q holds row r + q), and
  // at least two, so that the ring shifts become register renaming even
  // where one row is prefetched.
  constexpr int SU = PF > 1 ? PF : 2;
  const int su_end = ss_lo + (ss_hi - ss_lo) / SU * SU;
  for (; r < ss_lo; ++r) iter(r, std::false_type{}, Shift{}, Gen{});
  for (; r < su_end; r += SU) {
    static_for<SU>([&](auto q) {
      iter(r + q, std::true_type{}, std::integral_constant<int, decltype(q)::value % PF>{}, Gen{});
    });
  }
  for (; r < ss_hi; ++r) iter(r, std::true_type{}, Shift{}, Gen{});
  for (; r <= r_last; ++r) iter(r, std::false_type{}, Shift{}, Gen{});
}

// Strips that touch the grid's x-edges apply the mirror; interior strips skip it.
template <int MODEL, int STENCIL, int NS, int MODE, int K = 1, int GATE = 0, int HK = kHkAny, bool FR = true>
__device__ __forceinline__ void sweep_wave(const double* const* in, double* const* out,
                                           double* const (*ys)[kMaxFields], const KConst& c,
                                           int wid) {
  const int x0 = (wid / c.nby) * (kWave - 2 * K * NS) - K * NS;
  if constexpr (MODEL == RD_MODEL_BOCF) {
    if (strip_touches_edge(x0, c))
      sweep_wave_impl<MODEL, STENCIL, NS, MODE, true, K, GATE, HK, FR>(in, out, ys, c, wid);
    else
      sweep_wave_impl<MODEL, STENCIL, NS, MODE, false, K, GATE, HK, FR>(in, out, ys, c, wid);
  } else if (c.periodic) {  // no x-edge either: every strip wraps
    sweep_wave_impl<MODEL, STENCIL, NS, MODE, false, K, GATE, HK, FR, kBoundaryPeriodic>(in, out, ys, c, wid);
  } else if (strip_touches_edge(x0, c)) {
    sweep_wave_impl<MODEL, STENCIL, NS, MODE, true, K, GATE, HK, FR, kBoundaryNoFlux>(in, out, ys, c, wid);
  } else {
    sweep_wave_impl<MODEL, STENCIL, NS, MODE, false, K, GATE, HK, FR, kBoundaryNoFlux>(in, out, ys, c, wid);
  }
}

template <int MODEL, int STENCIL, int NS, int MODE, int K, int GATE, int HK>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(SweepOccupancy<MODEL, STENCIL, NS, MODE, K>::value)))
void sweep_kernel(SweepArgs a) {
  const int blk = xcd_order((int)blockIdx.x, (int)gridDim.x);
  const int wid = __builtin_amdgcn_readfirstlane(blk * (int)(blockDim.x / kWave) + (int)(threadIdx.x / kWave));
  if (wid >= a.c.nsx * a.c.nby) return;  // whole waves only: no barrier follows
  sweep_wave<MODEL, STENCIL, NS, MODE, K, GATE, HK>(a.in, a.out, a.ys, a.c, wid);
}

template <int MODEL, int STENCIL, int NS, int MODE, int K, int GATE, int HK>
hipError_t launch_sweep_k(const SweepArgs& a, hipStream_t stream) {
  const int waves = a.c.nsx * a.c.nby;
  const int blocks = (waves + kSweepWaves - 1) / kSweepWaves;
  hipLaunchKernelGGL((sweep_kernel<MODEL, STENCIL, NS, MODE, K, GATE, HK>), dim3(blocks), dim3(kSweepWaves * kWave), 0, stream,
                     a);
  return hipGetLastError();
}

// One step of a gate scheme (gated models, state or state and tangent).
template <int MODEL, int STENCIL, int MODE, int GATE, int HK>
hipError_t launch_sweep_gate(const SweepArgs& a, hipStream_t stream) {
  if constexpr (ModelTraits<MODEL>::GATED && MODE != kModeStages)
    return launch_sweep_k<MODEL, STENCIL, 1, MODE, 1, GATE, HK>(a, stream);
  return hipErrorInvalidValue;
}

// One launch of a.c.ksteps steps (1 unless MultiStep allows more).
template <int MODEL, int STENCIL, int NS, int MODE, int HK>
hipError_t launch_sweep(const SweepArgs& a, hipStream_t stream) {
  if (MODE == kModeStages && NS == 1) return hipSuccess;  // Euler has no inner stage
  constexpr int KMAX = MultiStep<MODEL, NS, MODE>::max;
  switch (a.c.ksteps) {
    case 1: return launch_sweep_k<MODEL, STENCIL, NS, MODE, 1, 0, HK>(a, stream);
    case 2: if constexpr (KMAX >= 2) return launch_sweep_k<MODEL, STENCIL, NS, MODE, 2, 0, HK>(a, stream); break;
    case 4: if constexpr (KMAX >= 4) return launch_sweep_k<MODEL, STENCIL, NS, MODE, 4, 0, HK>(a, stream); break;
    case 8: if constexpr (KMAX >= 8) return launch_sweep_k<MODEL, STENCIL, NS, MODE, 8, 0, HK>(a, stream); break;
  }
  return hipErrorInvalidValue;
}

// Dispatch over stencil and scheme for one model, mode and H_k evaluation.
template <int MODEL, int MODE, int HK>
hipError_t launch_sweep_model_hk(int stencil, int scheme, const SweepArgs& a, hipStream_t s) {
  switch (stencil) {
    case RD_LAP5:
      if (scheme == RD_SCHEME_EULER) return launch_sweep<MODEL, RD_LAP5, 1, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_sweep<MODEL, RD_LAP5, 2, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_sweep<MODEL, RD_LAP5, 4, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RUSH_LARSEN) return launch_sweep_gate<MODEL, RD_LAP5, MODE, 1, HK>(a, s);
      if (scheme == RD_SCHEME_IMPLICIT_EULER) return launch_sweep_gate<MODEL, RD_LAP5, MODE, 2, HK>(a, s);
      break;
    case RD_LAP9:
      if (scheme == RD_SCHEME_EULER) return launch_sweep<MODEL, RD_LAP9, 1, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_sweep<MODEL, RD_LAP9, 2, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_sweep<MODEL, RD_LAP9, 4, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RUSH_LARSEN) return launch_sweep_gate<MODEL, RD_LAP9, MODE, 1, HK>(a, s);
      if (scheme == RD_SCHEME_IMPLICIT_EULER) return launch_sweep_gate<MODEL, RD_LAP9, MODE, 2, HK>(a, s);
      break;
    case RD_LAP9_ANISO:
      if (scheme == RD_SCHEME_EULER) return launch_sweep<MODEL, RD_LAP9_ANISO, 1, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_sweep<MODEL, RD_LAP9_ANISO, 2, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_sweep<MODEL, RD_LAP9_ANISO, 4, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RUSH_LARSEN) return launch_sweep_gate<MODEL, RD_LAP9_ANISO, MODE, 1, HK>(a, s);
      if (scheme == RD_SCHEME_IMPLICIT_EULER) return launch_sweep_gate<MODEL, RD_LAP9_ANISO, MODE, 2, HK>(a, s);
      break;
  }
  return hipErrorInvalidValue;
}

// Models with H_k run the smooth or the sharp evaluation of it (HkEval),
// chosen by the call's step_k; the others have one set of kernels.
template <int MODEL, int MODE>
hipError_t launch_sweep_model(int stencil, int scheme, const SweepArgs& a, hipStream_t s) {
  if constexpr (ModelTraits<MODEL>::GATED) {
    return a.c.sharp ? launch_sweep_model_hk<MODEL, MODE, kHkSharp>(stencil, scheme, a, s)
                     : launch_sweep_model_hk<MODEL, MODE, kHkSmooth>(stencil, scheme, a, s);
  } else {
    return launch_sweep_model_hk<MODEL, MODE, kHkAny>(stencil, scheme, a, s);
  }
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
RD_DECLARE_SWEEP(fwd, fhn)
RD_DECLARE_SWEEP(tan, diffusion)
RD_DECLARE_SWEEP(tan, barkley)
RD_DECLARE_SWEEP(tan, fk)
RD_DECLARE_SWEEP(tan, bocf)
RD_DECLARE_SWEEP(tan, fhn)
RD_DECLARE_SWEEP(stg, diffusion)
RD_DECLARE_SWEEP(stg, barkley)
RD_DECLARE_SWEEP(stg, fk)
RD_DECLARE_SWEEP(stg, bocf)
RD_DECLARE_SWEEP(stg, fhn)
#undef RD_DECLARE_SWEEP
#define RD_DECLARE_PIPE(kind, model) \
  hipError_t launch_pipe_##kind##_##model(int stencil, int scheme, const SweepArgs& a, hipStream_t s);
RD_DECLARE_PIPE(fwd, diffusion)
RD_DECLARE_PIPE(fwd, barkley)
RD_DECLARE_PIPE(fwd, fk)
RD_DECLARE_PIPE(fwd, bocf)
RD_DECLARE_PIPE(fwd, fhn)
RD_DECLARE_PIPE(tan, diffusion)
RD_DECLARE_PIPE(tan, barkley)
RD_DECLARE_PIPE(tan, fk)
RD_DECLARE_PIPE(tan, bocf)
RD_DECLARE_PIPE(tan, fhn)
RD_DECLARE_PIPE(stg, diffusion)
RD_DECLARE_PIPE(stg, barkley)
RD_DECLARE_PIPE(stg, fk)
RD_DECLARE_PIPE(stg, bocf)
RD_DECLARE_PIPE(stg, fhn)
#undef RD_DECLARE_PIPE

// Dispatch over models.
hipError_t launch_sweep_mode(int mode, int model, int stencil, int scheme, const SweepArgs& a,
                             hipStream_t s);

}  // namespace rd
