// rd_adjoint_fused.h -- one reverse step of an explicit Runge-Kutta scheme
// (Heun, RK4) with the stage inputs recomputed inside the kernel: reads z_n
// and lambda_{n+1}, writes lambda_n.  The two-kernel path (stage-input sweep
// writing Y_2 .. Y_S to memory, then adjoint_kernel reading them) moves
// 2 n_v + 3 n_v (S - 1) more doubles per cell; here the forward stages run a
// few rows ahead of the reverse stages in the same sweep and hand each stage
// input over in registers.  For models with at most two fields (the register
// rings hold every field of every stage input for up to 2S - 1 rows).
//
// Decomposition as the sweep: one wavefront per 64-column strip and row band.
// Iteration r loads z row r and lambda row r - D (D = S - 2); forward stage s
// (1 <= s < S) runs on row r - s and produces Y_{s+1} there exactly as the
// stage-input sweep does; reverse stage j (S >= j >= 1) runs on row
// r - D - (S - j + 1) exactly as adjoint_kernel does, reading Y_j from the
// ring it was produced into 2S - 2j iterations earlier.  A stage input is valid
// one column further in from the strip ends per forward stage and each
// reverse stage narrows by one more, so a strip keeps 64 - 2 (2S - 2) output
// columns (52 for RK4).  Results equal the two-kernel path bit for bit.
#pragma once

#include "rd_adjoint.h"

namespace rd {

struct AdjFusedArgs {
  const double* z[kMaxFields];       // z_n
  const double* lam_in[kMaxFields];  // lambda_{n+1}
  double* lam_out[kMaxFields];       // lambda_n
  KConst c;
};

// Halo columns on each side of a strip in the fused reverse step of an `ns`-stage scheme.
inline int fused_adjoint_halo(int ns) { return 2 * ns - 2; }

template <int MODEL, int STENCIL, int NS, bool EDGE>
__device__ __forceinline__ void adjoint_fused_wave(const AdjFusedArgs& a, int wid) {
  static_assert(NS == 2 || NS == 4, "Runge-Kutta schemes with inner stages");
  constexpr int NV = ModelTraits<MODEL>::NV;
  constexpr int NDF = ModelTraits<MODEL>::NDIFF;
  static_assert(NV <= 2, "register rings sized for at most two fields");
  constexpr int H = 2 * NS - 2;   // halo columns
  constexpr int TX = kWave - 2 * H;
  constexpr int D = NS - 2;       // rows the reverse sweep trails the forward one
  constexpr int ZD = 2 * NS - 1;  // z ring depth: z(r - a), a = 0 .. 2S-2
  constexpr int YD = 2 * NS - 3 > 3 ? 2 * NS - 3 : 3;  // Y_s ring depth (ages 0 .. 2S-4, and 0..2 for stencils)
  constexpr int LR = (NS + 1 > 3) ? NS + 1 : 3;
  constexpr bool ANISO = STENCIL == RD_LAP9_ANISO;
  const KConst& c = a.c;

  const int lane = threadIdx.x & (kWave - 1);
  const int sx = wid / c.nby;
  const int by = wid % c.nby;
  const int gx = sx * TX - H + lane;
  const int cx = grid_index(gx, c.nx, c);
  const bool out_col = lane >= H && lane < H + TX && gx < c.nx;
  const Column col = make_column(gx, c, ANISO);
  const ColumnNb nb = ANISO ? make_column_nb(gx, c) : ColumnNb{0.0, 0.0};

  const int yA = by * c.ty;
  const int yB = min(yA + c.ty, c.ny);
  const int r_first = max(yA - (2 * NS - 2), 0);
  const int r_last = yB - 1 + 2 * NS - 2;
  const int z_end = min(yB + 2 * NS - 2, c.ny);  // z rows yA-(2S-2) .. yB+2S-3
  const int l_lo = max(yA - NS, 0), l_end = min(yB + NS, c.ny);  // lambda rows
  const size_t nx = (size_t)c.nx;

  double zr[ZD][NV];          // z at row r - a
  double yr[NS + 1][YD][NV];  // yr[s][a] = Y_s at row (r - s + 1) - a, s = 2 .. S
  double lr[LR][NV];          // lambda_{n+1} at row (r - D) - a
  double lacc[NS][NV];        // running lambda_n at row (r - D) - 1 - a
  double kbu[NS + 1][3][NDF]; // kbar_j diffusive components at rows rho_j + 1, rho_j, rho_j - 1
  double kbg[NS + 1][NV];     // kbar_j other components at row rho_j
  double kbgn[NS + 1][NV];    // ... produced this iteration
#pragma unroll
  for (int q = 0; q < ZD; ++q)
#pragma unroll
    for (int f = 0; f < NV; ++f) zr[q][f] = 0.0;
#pragma unroll
  for (int s = 0; s <= NS; ++s)
#pragma unroll
    for (int q = 0; q < YD; ++q)
#pragma unroll
      for (int f = 0; f < NV; ++f) yr[s][q][f] = 0.0;
#pragma unroll
  for (int q = 0; q < LR; ++q)
#pragma unroll
    for (int f = 0; f < NV; ++f) lr[q][f] = 0.0;
#pragma unroll
  for (int q = 0; q < NS; ++q)
#pragma unroll
    for (int f = 0; f < NV; ++f) lacc[q][f] = 0.0;
#pragma unroll
  for (int j = 0; j <= NS; ++j) {
#pragma unroll
    for (int f = 0; f < NV; ++f) kbg[j][f] = kbgn[j][f] = 0.0;
#pragma unroll
    for (int d = 0; d < NDF; ++d) kbu[j][0][d] = kbu[j][1][d] = kbu[j][2][d] = 0.0;
  }

  // Rows loaded ahead, as many as the steady run is unrolled: when iteration r
  // starts, zpre[p] holds z row r + p and lpre[p] lambda row (r - D) + p (the
  // first lambda row is the band's l_lo, taken when r - D reaches it); loads
  // past a range end re-read its last row.
  constexpr int kAhead = NS == 2 ? 4 : 2;
  double zpre[kAhead][NV], lpre[kAhead][NV];
#pragma unroll
  for (int p = 0; p < kAhead; ++p)
#pragma unroll
    for (int f = 0; f < NV; ++f) zpre[p][f] = lpre[p][f] = 0.0;
  if (r_first < z_end) {
#pragma unroll
    for (int p = 0; p < kAhead; ++p)
#pragma unroll
      for (int f = 0; f < NV; ++f) zpre[p][f] = a.z[f][(size_t)min(r_first + p, z_end - 1) * nx + cx];
  }
  if (l_lo < l_end) {
#pragma unroll
    for (int p = 0; p < kAhead; ++p)
#pragma unroll
      for (int f = 0; f < NV; ++f) lpre[p][f] = a.lam_in[f][(size_t)min(l_lo + p, l_end - 1) * nx + cx];
  }

  // One iteration: take z row r and lambda row r - D, run the forward stages
  // on rows r - s and the reverse stages on rows r - D - (S - j + 1).  STEADY
  // marks iterations in which every stage is active and no stage row touches
  // the y-edges: no branch, no mirror, and the stores need no row test, so the
  // stages' independent work forms one basic block.  Loads past a range end
  // re-read its last row (in bounds, never used).  PHASE = 1 + i: ramp-up
  // iteration i (row yA - (2S - 2) + i) of a band away from the y-edges, where
  // which stages run is known at compile time: lambda from i = 2S - 4, forward
  // stage s from i = 2s, reverse stage j from i = 4S - 2j - 2 (never j = 1);
  // like the steady ones, such iterations test no ranges and apply no mirror.
  // SLOT < 0: the prefetch rings shift by one row and this iteration loads
  // the row kAhead ahead; SLOT = q: iteration q of an unrolled steady block,
  // whose rows slot q holds (the block loads the next block's rows itself).
  auto iter = [&](int r, auto steady_tag, auto phase_tag, auto slot_tag) __attribute__((always_inline)) {
    constexpr bool STEADY = decltype(steady_tag)::value;
    constexpr int SLOT = decltype(slot_tag)::value;
    constexpr int Q = SLOT < 0 ? 0 : SLOT;
    constexpr int PHASE = STEADY ? 0 : decltype(phase_tag)::value;
    constexpr bool UP = PHASE > 0;
    constexpr bool FIXED = STEADY || UP;
    // advance the rings by one row
#pragma unroll
    for (int q = ZD - 1; q > 0; --q)
#pragma unroll
      for (int f = 0; f < NV; ++f) zr[q][f] = zr[q - 1][f];
#pragma unroll
    for (int s = 2; s <= NS; ++s)
#pragma unroll
      for (int q = YD - 1; q > 0; --q)
#pragma unroll
        for (int f = 0; f < NV; ++f) yr[s][q][f] = yr[s][q - 1][f];
#pragma unroll
    for (int q = LR - 1; q > 0; --q)
#pragma unroll
      for (int f = 0; f < NV; ++f) lr[q][f] = lr[q - 1][f];
#pragma unroll
    for (int q = NS - 1; q > 0; --q)
#pragma unroll
      for (int f = 0; f < NV; ++f) lacc[q][f] = lacc[q - 1][f];
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
    // z row r and lambda row r - D (rows outside their ranges are never read)
    if (FIXED || r < z_end) {
#pragma unroll
      for (int f = 0; f < NV; ++f) zr[0][f] = zpre[Q][f];
      if constexpr (SLOT < 0) {
#pragma unroll
        for (int p = 0; p + 1 < kAhead; ++p)
#pragma unroll
          for (int f = 0; f < NV; ++f) zpre[p][f] = zpre[p + 1][f];
        const size_t o = (size_t)min(r + kAhead, z_end - 1) * nx + cx;
#pragma unroll
        for (int f = 0; f < NV; ++f) zpre[kAhead - 1][f] = a.z[f][o];
      }
    }
    const int lrow = r - D;
    if (STEADY || (UP ? PHASE - 1 >= 2 * NS - 4 : (lrow >= l_lo && lrow < l_end))) {
#pragma unroll
      for (int f = 0; f < NV; ++f) lr[0][f] = lpre[Q][f];
      if constexpr (SLOT < 0) {
#pragma unroll
        for (int p = 0; p + 1 < kAhead; ++p)
#pragma unroll
          for (int f = 0; f < NV; ++f) lpre[p][f] = lpre[p + 1][f];
        const size_t o = (size_t)min(lrow + kAhead, l_end - 1) * nx + cx;
#pragma unroll
        for (int f = 0; f < NV; ++f) lpre[kAhead - 1][f] = a.lam_in[f][o];
      }
    }

    // forward stages: stage s on row r - s produces Y_{s+1} there
#pragma unroll
    for (int s = 1; s < NS; ++s) {
      const int rho = r - s;
      if (UP) {
        if (PHASE - 1 < 2 * s) continue;  // folded
      } else if (!STEADY) {
        const int ext = 2 * NS - 2 - s;
        if (rho < max(yA - ext, 0) || rho >= min(yB + ext, c.ny)) continue;  // wave-uniform
      }
      double y[NV], up[NDF], dn[NDF];
      if (s == 1) {
#pragma unroll
        for (int f = 0; f < NV; ++f) y[f] = zr[1][f];
#pragma unroll
        for (int d = 0; d < NDF; ++d) {
          up[d] = zr[2][d];
          dn[d] = zr[0][d];
        }
      } else {
#pragma unroll
        for (int f = 0; f < NV; ++f) y[f] = yr[s][1][f];
#pragma unroll
        for (int d = 0; d < NDF; ++d) {
          up[d] = yr[s][2][d];
          dn[d] = yr[s][0][d];
        }
      }
      if (!FIXED) {
#pragma unroll
        for (int d = 0; d < NDF; ++d) {
          if (rho == 0) up[d] = y[d];
          if (rho == c.ny - 1) dn[d] = y[d];
        }
      }
      double lap[NDF];
#pragma unroll
      for (int d = 0; d < NDF; ++d)
        lap[d] = diffusion<STENCIL, EDGE, !FIXED>(up[d], y[d], dn[d], col, rho, c, c.dcoef[d]);
      double kr[NV];
      eval_rates<MODEL, false>(c, y, kr);
#pragma unroll
      for (int d = 0; d < NDF; ++d) kr[d] = lap[d] + kr[d];
      const double cs = Scheme<NS>::next_coef(c, s);
#pragma unroll
      for (int f = 0; f < NV; ++f) yr[s + 1][0][f] = zr[s][f] + cs * kr[f];
    }

    // reverse stages: stage j on row (r - D) - (S - j + 1)
#pragma unroll
    for (int j = NS; j >= 1; --j) {
      const int lag = NS - j + 1;
      const int rho = r - D - lag;
      if (UP) {
        if (PHASE - 1 < 4 * NS - 2 * j - 2) continue;  // folded
      } else if (!STEADY && (rho < max(yA - (j - 1), 0) || rho >= min(yB + (j - 1), c.ny))) {
        continue;  // wave-uniform
      }

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
        if (!FIXED) {
          if (rho == 0) up[d] = kb[d];
          if (rho == c.ny - 1) dn[d] = kb[d];
        }
        if constexpr (ANISO)
          lapT[d] = flux_transpose<EDGE, !FIXED>(up[d], kb[d], dn[d], col, nb, rho, c, c.dcoef[d]);
        else
          lapT[d] = diffusion<STENCIL, EDGE, !FIXED>(up[d], kb[d], dn[d], col, rho, c, c.dcoef[d]);
      }
      // Y_j at row rho: z for j = 1 (age 2S - 2), else produced 2S - 2j iterations ago
      double y[NV];
#pragma unroll
      for (int f = 0; f < NV; ++f) y[f] = j == 1 ? zr[2 * NS - 2][f] : yr[j][2 * NS - 2 * j][f];
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
      } else if (out_col && (FIXED || (rho >= yA && rho < yB))) {
        const size_t oo = (size_t)rho * nx + gx;
#pragma unroll
        for (int f = 0; f < NV; ++f) a.lam_out[f][oo] = lacc[lag - 1][f];
      }
    }
  };

  // Steady iterations: r >= yA + 2S - 2 and r >= 2S - 1 (the last reverse
  // stage's row is in the band and not row 0), r < min(yB + 2S - 2, ny) (the
  // first forward stage's row is not row ny - 1 and every stage's row is
  // before its range end).  The steady run goes kUnroll rows at a time, so the
  // ring shifts become register renaming inside the unrolled body.
  constexpr int kUnroll = kAhead;
  using Shift = std::integral_constant<int, -1>;
  const int ss_lo = min(max(yA + 2 * NS - 2, 2 * NS - 1), r_last + 1);
  const int ss_hi = max(min(yB + 2 * NS - 2, c.ny), ss_lo);
  const int ss_end = ss_lo + (ss_hi - ss_lo) / kUnroll * kUnroll;
  using Gen = std::integral_constant<int, 0>;
  // Fixed ramp-up: r_first = yA - (2S - 2) and ss_lo = yA + 2S - 2, and every
  // stage row of the ramp lies at least one row inside both y-edges.
  const bool fixed_up = yA >= 2 * NS - 2 && yA + 4 * NS < c.ny;
  int r = r_first;
  if (fixed_up) {
    static_for<4 * NS - 4>([&](auto i) {
      constexpr int I = decltype(i)::value;
      iter(r_first + I, std::false_type{}, std::integral_constant<int, 1 + I>{}, Shift{});
    });
    r = ss_lo;
  }
  for (; r < ss_lo; ++r) iter(r, std::false_type{}, Gen{}, Shift{});
  for (; r < ss_end; r += kUnroll) {
    // the next block's rows, issued before this block's arithmetic: the copy
    // into the slots at the end of the block then finds them landed (the
    // compiler does not keep loaded registers in place across the back edge)
    double nz[kAhead][NV], nl[kAhead][NV];
#pragma unroll
    for (int q = 0; q < kAhead; ++q) {
      const size_t oz = (size_t)min(r + kAhead + q, z_end - 1) * nx + cx;
      const size_t ol = (size_t)min(r - D + kAhead + q, l_end - 1) * nx + cx;
#pragma unroll
      for (int f = 0; f < NV; ++f) {
        nz[q][f] = a.z[f][oz];
        nl[q][f] = a.lam_in[f][ol];
      }
    }
    static_for<kUnroll>([&](auto q) { iter(r + q, std::true_type{}, Gen{}, q); });
#pragma unroll
    for (int q = 0; q < kAhead; ++q)
#pragma unroll
      for (int f = 0; f < NV; ++f) {
        zpre[q][f] = nz[q][f];
        lpre[q][f] = nl[q][f];
      }
  }
  for (; r < ss_hi; ++r) iter(r, std::true_type{}, Gen{}, Shift{});
  for (; r <= r_last; ++r) iter(r, std::false_type{}, Gen{}, Shift{});
}

template <int MODEL, int STENCIL, int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void adjoint_fused_kernel(AdjFusedArgs a) {
  const int blk = xcd_order((int)blockIdx.x, (int)gridDim.x);
  const int wid = __builtin_amdgcn_readfirstlane(blk * (int)(blockDim.x / kWave) + (int)(threadIdx.x / kWave));
  if (wid >= a.c.nsx * a.c.nby) return;  // whole waves only: no barrier follows
  constexpr int H = 2 * NS - 2;
  if (strip_touches_edge((wid / a.c.nby) * (kWave - 2 * H) - H, a.c))
    adjoint_fused_wave<MODEL, STENCIL, NS, true>(a, wid);
  else
    adjoint_fused_wave<MODEL, STENCIL, NS, false>(a, wid);
}

template <int MODEL, int STENCIL, int NS>
hipError_t launch_adjoint_fused(const AdjFusedArgs& a, hipStream_t stream) {
  const int waves = a.c.nsx * a.c.nby;
  const int blocks = (waves + 3) / 4;
  hipLaunchKernelGGL((adjoint_fused_kernel<MODEL, STENCIL, NS>), dim3(blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

// Models with at most two fields, no-flux boundaries, Heun or RK4.
template <int MODEL>
hipError_t launch_adjoint_fused_model(int stencil, int scheme, const AdjFusedArgs& a, hipStream_t s) {
  if constexpr (ModelTraits<MODEL>::NV <= 2) {
    switch (stencil) {
      case RD_LAP5:
        if (scheme == RD_SCHEME_HEUN) return launch_adjoint_fused<MODEL, RD_LAP5, 2>(a, s);
        if (scheme == RD_SCHEME_RK4) return launch_adjoint_fused<MODEL, RD_LAP5, 4>(a, s);
        break;
      case RD_LAP9:
        if (scheme == RD_SCHEME_HEUN) return launch_adjoint_fused<MODEL, RD_LAP9, 2>(a, s);
        if (scheme == RD_SCHEME_RK4) return launch_adjoint_fused<MODEL, RD_LAP9, 4>(a, s);
        break;
      case RD_LAP9_ANISO:
        if (scheme == RD_SCHEME_HEUN) return launch_adjoint_fused<MODEL, RD_LAP9_ANISO, 2>(a, s);
        if (scheme == RD_SCHEME_RK4) return launch_adjoint_fused<MODEL, RD_LAP9_ANISO, 4>(a, s);
        break;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint_fused_diffusion(int stencil, int scheme, const AdjFusedArgs& a, hipStream_t s);
hipError_t launch_adjoint_fused_barkley(int stencil, int scheme, const AdjFusedArgs& a, hipStream_t s);
hipError_t launch_adjoint_fused_fhn(int stencil, int scheme, const AdjFusedArgs& a, hipStream_t s);

}  // namespace rd
