// rd_tune.cpp -- band-height autotuner.
//
// The rows per wavefront band trade parallelism (more, shorter bands keep more
// waves in flight) against redundant work (each band end recomputes a ramp of
// NS rows per stage).  The best value depends on grid shape, model, stencil
// and scheme, so the first call for each such key times a set of candidates
// with HIP events on the caller's stream -- trial launches read the caller's
// state and write only workspace -- and caches the fastest.  Results do not
// depend on the choice (every band height computes identical bits).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "rd_host.h"
#include "rd_sweep.h"

namespace rd {

namespace {
std::mutex g_mu;
// Keyed by the problem and by the overrides in force: a fixed variant, band
// height or step count restricts the candidates, so it selects its own entry.
using Key = std::tuple<int, int, int, int, int, int, int, int, int, int>;
std::map<Key, Plan> g_cache;
bool g_enabled = true;
int g_override = -1;          // rows per band (> 0: fixed)
int g_variant_override = -1;  // kernel variant (>= 0: fixed)
int g_ksteps_override = -1;   // steps per launch (> 0: fixed, capped by the model's maximum)
}  // namespace

void set_ksteps_override(int k) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_ksteps_override = k;
}

void set_tile_rows_override(int rows) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_override = rows;
}

void set_variant_override(int variant) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_variant_override = variant;
}

void set_autotune(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_enabled = on;
}

// SIMDs of the current device (CUs x 4), queried once per process.
static int simd_count() {
  static const int n = [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    return 4 * cus;
  }();
  return n;
}

int heuristic_rows(int nx, int ny, int ns) {
  const int tx = 64 - 2 * ns;
  const int nsx = (nx + tx - 1) / tx;
  const int target_waves = 2048;
  const int nby = (target_waves + nsx - 1) / nsx;
  int ty = (ny + nby - 1) / nby;
  if (ty < 2 * ns) ty = 2 * ns;
  return ty < ny ? ty : ny;
}

// Starting plan without measurements: the pipelined kernel with bands sized
// for about 640 workgroups, or the sweep kernel when the variant is fixed to it.
static Plan heuristic_plan(int nx, int ny, int ns, int variant) {
  if (variant == kVariantSweep) return Plan{kVariantSweep, heuristic_rows(nx, ny, ns)};
  const int tx = 64 - 2 * ns;
  const int nsx = (nx + tx - 1) / tx;
  const int nby = (640 + nsx - 1) / nsx;
  int ty = (ny + nby - 1) / nby;
  if (ty < 4 * ns) ty = 4 * ns;
  return Plan{kVariantPipe, ty < ny ? ty : ny};
}

// Steps per launch a fixed override asks for, within [1, kmax].
static int fixed_k(int kmax) {
  if (g_ksteps_override <= 0) return 0;
  return g_ksteps_override < kmax ? g_ksteps_override : kmax;
}

static Plan apply_overrides(Plan p, int ny, int kmax) {
  if (g_variant_override >= 0) p.variant = g_variant_override;
  if (g_override > 0) p.ty = g_override < ny ? g_override : ny;
  // several steps per launch exist only in the sweep kernel
  if (fixed_k(kmax) > 1 && g_variant_override != kVariantPipe) p.variant = kVariantSweep;
  if (fixed_k(kmax) > 0 && p.variant == kVariantSweep) p.k = fixed_k(kmax);
  return p;
}

Plan tuned_plan(int kind, int model, int stencil, int scheme, int nx, int ny, int ns, hipStream_t s,
                const std::function<hipError_t(Plan)>& trial, bool allow_pipe, int shape_key,
                int fallback_ty, int kmax) {
  bool tune;
  Plan fallback;
  std::vector<Plan> cands;
  Key key;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const int vfix = allow_pipe ? g_variant_override : kVariantSweep;
    const int kfix = fixed_k(kmax);
    key = Key(kind, model, stencil, scheme, nx, ny, vfix, g_override > 0 ? g_override : 0, shape_key,
              kmax > 1 ? kfix : 1);
    Plan start = heuristic_plan(nx, ny, ns, vfix);
    if (fallback_ty > 0) start.ty = fallback_ty < ny ? fallback_ty : ny;
    fallback = apply_overrides(start, ny, kmax);
    if (!allow_pipe) fallback.variant = kVariantSweep;
    if (g_override > 0 && vfix >= 0 && (kmax == 1 || kfix > 0)) return fallback;  // fully fixed
    auto it = g_cache.find(key);
    if (it != g_cache.end()) return it->second;
    tune = g_enabled;
    if (vfix != kVariantPipe)
      for (int k : {1, 2, 4, 8}) {
        if (k > kmax || (kfix > 0 && k != kfix)) continue;
        std::vector<int> tys = {2, 3, 4, 6, 8, 10, 12, 16, 24, 32, 48, 64};
        // Band heights whose wave count just fits m rounds of one wave per
        // SIMD: a partly filled last round costs as much as a full one.
        const int nsx = (nx + strip_width(ns * k) - 1) / strip_width(ns * k);
        for (int m = 1; m <= 12; ++m) {
          const int nby = m * simd_count() / nsx;
          if (nby >= 1) tys.push_back((ny + nby - 1) / nby);
        }
        std::sort(tys.begin(), tys.end());
        tys.erase(std::unique(tys.begin(), tys.end()), tys.end());
        for (int ty : tys)
          if (ty <= ny && ty >= ns && ty <= 256 && (g_override <= 0 || ty == fallback.ty))
            cands.push_back(Plan{kVariantSweep, ty, k});
      }
    if (allow_pipe && vfix != kVariantSweep && kfix <= 1)
      for (int ty : {4, 6, 8, 12, 16, 24, 32, 48, 64, 96})
        if (ty <= ny && ty >= ns && (g_override <= 0 || ty == fallback.ty)) cands.push_back(Plan{kVariantPipe, ty});
  }
  if (!tune) return fallback;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
    return fallback;  // no timing inside a graph capture
  if (cands.empty()) cands.push_back(fallback);

  // Two passes over the candidates, keeping each one's faster pass: the
  // first pass (three launches each) also brings the clocks up, which would
  // otherwise favour the candidates timed last; the second repeats each
  // candidate for about 0.3 ms (3 to 50 launches), so that short launches
  // are not ranked by timer noise.
  hipEvent_t e0 = nullptr, e1 = nullptr;
  Plan best = fallback;
  bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  if (ok) ok = trial(fallback) == hipSuccess;  // warm-up
  std::vector<float> per_step(cands.size(), 1e30f);
  for (int pass = 0; pass < 2; ++pass)
    for (size_t i = 0; ok && i < cands.size(); ++i) {
      const float launch_ms = per_step[i] * (float)cands[i].k;
      const int reps = pass == 0 ? 3 : std::max(3, std::min(50, (int)(0.3f / std::max(launch_ms, 1e-3f)) + 1));
      ok = hipEventRecord(e0, s) == hipSuccess;
      for (int r = 0; ok && r < reps; ++r) ok = trial(cands[i]) == hipSuccess;
      ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
      float ms = 0.f;
      ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
      if (ok) per_step[i] = std::min(per_step[i], ms / (float)cands[i].k);
    }
  // Near-ties (within 2%, about the run-to-run noise) go to the first
  // candidate in list order, so that repeated tunings pick the same plan.
  float best_ms = 1e30f;
  for (size_t i = 0; ok && i < cands.size(); ++i) best_ms = std::min(best_ms, per_step[i]);
  for (size_t i = 0; ok && i < cands.size(); ++i)
    if (per_step[i] <= best_ms * 1.02f) {
      best = cands[i];
      break;
    }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (!ok) {
    (void)hipGetLastError();
    return fallback;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[key] = best;
  return best;
}

int tuned_rows(int kind, int model, int stencil, int scheme, int nx, int ny, int ns, hipStream_t s,
               const std::function<hipError_t(int)>& trial, int shape_key, int fallback_ty) {
  return tuned_plan(kind, model, stencil, scheme, nx, ny, ns, s,
                    [&](Plan p) { return trial(p.ty); }, false, shape_key, fallback_ty).ty;
}

Plan current_plan(int kind, int model, int stencil, int scheme, int nx, int ny, int ns, bool allow_pipe,
                  int kmax) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int vfix = allow_pipe ? g_variant_override : kVariantSweep;
  auto it = g_cache.find(Key(kind, model, stencil, scheme, nx, ny, vfix, g_override > 0 ? g_override : 0, 0,
                             kmax > 1 ? fixed_k(kmax) : 1));
  if (it != g_cache.end()) return it->second;
  Plan p = apply_overrides(heuristic_plan(nx, ny, ns, vfix), ny, kmax);
  if (!allow_pipe) p.variant = kVariantSweep;
  return p;
}

int current_rows(int kind, int model, int stencil, int scheme, int nx, int ny, int ns) {
  return current_plan(kind, model, stencil, scheme, nx, ny, ns, false).ty;
}

}  // namespace rd

extern "C" {

int rd_set_kernel_variant(int32_t variant) {
  if (variant > rd::kVariantPipe) return rd::fail(RD_EINVAL, "unknown kernel variant %d", variant);
  rd::set_variant_override(variant < 0 ? -1 : variant);
  return RD_OK;
}

int rd_get_plan(const rd_problem* p, int32_t op, int32_t* variant, int32_t* rows) {
  int rc = rd::validate(p);
  if (rc) return rc;
  if (rd::is_3d(p->stencil)) return rd::fail(RD_EUNSUPPORTED, "3-D grids have a fixed launch shape (no plan)");
  if (!rows || !variant) return rd::fail(RD_EINVAL, "output pointer is NULL");
  int kind;
  switch (op) {
    case RD_OP_STEP: kind = rd::kTuneForward; break;
    case RD_OP_JVP: kind = rd::kTuneTangent; break;
    default: return rd::fail(RD_EINVAL, "rd_get_plan: op %d has no single-grid plan", op);
  }
  const int ns = rd::n_stages(p->scheme);
  const rd::Plan pl = rd::current_plan(kind, p->model, p->stencil, p->scheme, p->nx, p->ny, ns, true,
                                       op == RD_OP_STEP ? rd::max_steps_per_launch(p->model, ns) : 1);
  *variant = pl.variant;
  *rows = pl.ty;
  return RD_OK;
}

int rd_get_steps_per_launch(const rd_problem* p, int32_t* steps) {
  int rc = rd::validate(p);
  if (rc) return rc;
  if (rd::is_3d(p->stencil)) return rd::fail(RD_EUNSUPPORTED, "3-D grids have a fixed launch shape (no plan)");
  if (!steps) return rd::fail(RD_EINVAL, "steps is NULL");
  const int ns = rd::n_stages(p->scheme);
  *steps = rd::current_plan(rd::kTuneForward, p->model, p->stencil, p->scheme, p->nx, p->ny, ns, true,
                            rd::max_steps_per_launch(p->model, ns)).k;
  return RD_OK;
}

int rd_set_steps_per_launch(int32_t steps) {
  if (steps > 0 && steps != 1 && steps != 2 && steps != 4 && steps != 8)
    return rd::fail(RD_EINVAL, "steps per launch %d is not 1, 2, 4 or 8", steps);
  rd::set_ksteps_override(steps > 0 ? steps : -1);
  return RD_OK;
}

int rd_get_tile_rows(const rd_problem* p, int32_t op, int32_t* rows) {
  int rc = rd::validate(p);
  if (rc) return rc;
  if (rd::is_3d(p->stencil)) return rd::fail(RD_EUNSUPPORTED, "3-D grids have a fixed launch shape (no plan)");
  if (!rows) return rd::fail(RD_EINVAL, "rows is NULL");
  int kind;
  switch (op) {
    case RD_OP_STEP: kind = rd::kTuneForward; break;
    case RD_OP_JVP: kind = rd::kTuneTangent; break;
    case RD_OP_VJP: kind = rd::kTuneAdjoint; break;
    default: return rd::fail(RD_EINVAL, "rd_get_tile_rows: op %d has no single-grid band height", op);
  }
  const int ns = rd::n_stages(p->scheme);
  if (op == RD_OP_VJP && rd::fused_adjoint(p)) {  // the fused reverse step's own band height
    *rows = rd::current_rows(rd::kTuneAdjointFused, p->model, p->stencil, p->scheme, p->nx, p->ny, 2 * ns - 2);
    return RD_OK;
  }
  *rows = op == RD_OP_VJP ? rd::current_rows(kind, p->model, p->stencil, p->scheme, p->nx, p->ny, ns)
                          : rd::current_plan(kind, p->model, p->stencil, p->scheme, p->nx, p->ny, ns, true,
                                             op == RD_OP_STEP ? rd::max_steps_per_launch(p->model, ns) : 1).ty;
  return RD_OK;
}

int rd_set_tile_rows(int32_t rows) {
  rd::set_tile_rows_override(rows);
  return RD_OK;
}

int rd_set_autotune(int32_t enable) {
  rd::set_autotune(enable != 0);
  return RD_OK;
}

}  // extern "C"
