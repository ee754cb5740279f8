// rd_batch.h -- one fused step of many independent problems (an ensemble or a
// set of Krylov directions) on grids of different sizes, in a single launch.
//
// Every instance is cut into 64-column strips and row bands exactly as a
// single-grid launch would cut it; the waves of all instances are numbered
// consecutively and each wave looks its instance up in a device-side table
// (binary search over the first wave of each instance, in scalar registers),
// then runs the same per-wave sweep as rd_step / rd_jvp.  Results are
// therefore bit-identical to per-instance calls.
//
// The table is written by a small setup kernel that receives the instance
// descriptors as kernel arguments, so no host buffer has to outlive the call
// and the whole sequence consists of kernel launches only.
#pragma once

#include "rd_sweep.h"

namespace rd {

struct BatchInst {
  double* a[kMaxPacked];  // caller's arrays: state fields, then tangent fields
  double* b[kMaxPacked];  // equally sized workspace arrays (ping-pong partner)
  double dt, h2, h6;      // this instance's time step, dt/2, dt/6
  int nx, ny, nsx, nby, ty;
  int wave_begin;         // first global wave of this instance
};

constexpr int kInstPerSetup = 20;  // descriptors per setup launch (< 4 KiB of arguments)

struct BatchSetupArgs {
  BatchInst inst[kInstPerSetup];
  BatchInst* table;
  int first, count;
};
static_assert(sizeof(BatchSetupArgs) <= 4096, "kernel arguments are limited to 4 KiB");

struct BatchArgs {
  const BatchInst* table;
  int ninst;
  int total_waves;
  int parity;   // 0: a -> b, 1: b -> a
  int nf;       // arrays per instance
  KConst c;     // shared physics; grid fields and time steps come from the table
};

struct BatchCopyArgs {
  const BatchInst* table;
  int nf;
};

__global__ void batch_setup_kernel(BatchSetupArgs a);
__global__ void batch_copy_kernel(BatchCopyArgs a);

template <int MODEL, int STENCIL, int NS, int MODE, int GATE, int HK>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(SweepOccupancy<MODEL, STENCIL, NS, MODE>::value)))
void batch_sweep_kernel(BatchArgs a) {
  constexpr int NF = (MODE == kModeTangent ? 2 : 1) * ModelTraits<MODEL>::NV;
  const int blk = xcd_order((int)blockIdx.x, (int)gridDim.x);
  const int wid = __builtin_amdgcn_readfirstlane(blk * (int)(blockDim.x / kWave) + (int)(threadIdx.x / kWave));
  if (wid >= a.total_waves) return;  // whole waves only: no barrier follows
  int lo = 0, hi = a.ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.table[mid].wave_begin <= wid) lo = mid;
    else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const BatchInst& I = a.table[lo];
  KConst c = a.c;
  c.nx = I.nx;
  c.ny = I.ny;
  c.nsx = I.nsx;
  c.nby = I.nby;
  c.ty = I.ty;
  c.n_total = (double)I.nx;
  c.dt = I.dt;
  c.h2 = I.h2;
  c.h6 = I.h6;
  const double* in[kMaxPacked];
  double* out[kMaxPacked];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    in[f] = a.parity ? I.b[f] : I.a[f];
    out[f] = a.parity ? I.a[f] : I.b[f];
  }
  double* const no_stages[3][kMaxFields] = {};
  // The tangent step keeps the former loop structure: with the compile-time
  // ramps and the two-row steady unroll (a third more code) it measured 8-12%
  // slower here, although the single-grid tangent step gains from them.
  sweep_wave<MODEL, STENCIL, NS, MODE, 1, GATE, HK, MODE != kModeTangent>(in, out, no_stages, c, wid - I.wave_begin);
}

template <int MODEL, int STENCIL, int NS, int MODE, int HK, int GATE = 0>
hipError_t launch_batch(const BatchArgs& a, hipStream_t stream) {
  if constexpr (GATE != 0 && !ModelTraits<MODEL>::GATED) {
    return hipErrorInvalidValue;
  } else {
    const int blocks = (a.total_waves + 3) / 4;
    hipLaunchKernelGGL((batch_sweep_kernel<MODEL, STENCIL, NS, MODE, GATE, HK>), dim3(blocks), dim3(256), 0,
                       stream, a);
    return hipGetLastError();
  }
}

template <int MODEL, int MODE, int HK>
hipError_t launch_batch_model_hk(int stencil, int scheme, const BatchArgs& a, hipStream_t s) {
  switch (stencil) {
    case RD_LAP5:
      if (scheme == RD_SCHEME_EULER) return launch_batch<MODEL, RD_LAP5, 1, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_batch<MODEL, RD_LAP5, 2, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_batch<MODEL, RD_LAP5, 4, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RUSH_LARSEN) return launch_batch<MODEL, RD_LAP5, 1, MODE, HK, 1>(a, s);
      if (scheme == RD_SCHEME_IMPLICIT_EULER) return launch_batch<MODEL, RD_LAP5, 1, MODE, HK, 2>(a, s);
      break;
    case RD_LAP9:
      if (scheme == RD_SCHEME_EULER) return launch_batch<MODEL, RD_LAP9, 1, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_batch<MODEL, RD_LAP9, 2, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_batch<MODEL, RD_LAP9, 4, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RUSH_LARSEN) return launch_batch<MODEL, RD_LAP9, 1, MODE, HK, 1>(a, s);
      if (scheme == RD_SCHEME_IMPLICIT_EULER) return launch_batch<MODEL, RD_LAP9, 1, MODE, HK, 2>(a, s);
      break;
    case RD_LAP9_ANISO:
      if (scheme == RD_SCHEME_EULER) return launch_batch<MODEL, RD_LAP9_ANISO, 1, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_HEUN) return launch_batch<MODEL, RD_LAP9_ANISO, 2, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RK4) return launch_batch<MODEL, RD_LAP9_ANISO, 4, MODE, HK>(a, s);
      if (scheme == RD_SCHEME_RUSH_LARSEN) return launch_batch<MODEL, RD_LAP9_ANISO, 1, MODE, HK, 1>(a, s);
      if (scheme == RD_SCHEME_IMPLICIT_EULER) return launch_batch<MODEL, RD_LAP9_ANISO, 1, MODE, HK, 2>(a, s);
      break;
  }
  return hipErrorInvalidValue;
}

// Models with H_k run the smooth or the sharp evaluation of it, chosen by the
// batch's step_k (the same kernels as rd_step / rd_jvp).
template <int MODEL, int MODE>
hipError_t launch_batch_model(int stencil, int scheme, const BatchArgs& a, hipStream_t s) {
  if constexpr (ModelTraits<MODEL>::GATED) {
    return a.c.sharp ? launch_batch_model_hk<MODEL, MODE, kHkSharp>(stencil, scheme, a, s)
                     : launch_batch_model_hk<MODEL, MODE, kHkSmooth>(stencil, scheme, a, s);
  } else {
    return launch_batch_model_hk<MODEL, MODE, kHkAny>(stencil, scheme, a, s);
  }
}

#define RD_DECLARE_BATCH(model)                                                           \
  hipError_t launch_batch_##model(bool tangent, int stencil, int scheme, const BatchArgs& a, \
                                  hipStream_t s);
RD_DECLARE_BATCH(diffusion)
RD_DECLARE_BATCH(barkley)
RD_DECLARE_BATCH(fk)
RD_DECLARE_BATCH(bocf)
RD_DECLARE_BATCH(fhn)
#undef RD_DECLARE_BATCH

}  // namespace rd
