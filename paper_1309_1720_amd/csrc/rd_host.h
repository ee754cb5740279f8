// rd_host.h -- host-side helpers shared by the C ABI implementation files.
#pragma once

#include <functional>

#include "rd_device.h"

namespace rd {

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int n_fields(int model);
int n_params(int model);
int n_stages(int scheme);
bool gate_scheme(int scheme);  // Rush-Larsen or implicit Euler
int validate(const rd_problem* p);
int validate_fields(const rd_problem* p, double* const* f, const char* what);
void derive_constants(const rd_problem* p, KConst& c);
// Strips and bands for `halo` = stages per launch (NS times steps per launch).
void set_geometry(KConst& c, int halo, int ty);

// Autotuned rows per wave band (rd_tune.cpp).  `trial(ty)` enqueues one
// launch with that band height that writes only workspace.
enum TuneKind { kTuneForward = 0, kTuneTangent = 1, kTuneAdjoint = 2, kTuneBatched = 3, kTuneAdjointFused = 20 };
struct Plan {
  int variant;  // StepVariant
  int ty;       // rows per band
  int k = 1;    // steps per launch (state-only sweep)
};
// Largest steps-per-launch the state-only sweep supports for this model and
// scheme (1: none).
int max_steps_per_launch(int model, int ns);
// Tunes kernel variant and band height together (trial launches write only
// workspace); allow_pipe = false restricts to the sweep kernel.  shape_key
// distinguishes launches whose grids nx x ny do not describe (batches);
// fallback_ty > 0 replaces the single-grid heuristic's band height.
Plan tuned_plan(int kind, int model, int stencil, int scheme, int nx, int ny, int ns, hipStream_t s,
                const std::function<hipError_t(Plan)>& trial, bool allow_pipe, int shape_key = 0,
                int fallback_ty = 0, int kmax = 1);
Plan current_plan(int kind, int model, int stencil, int scheme, int nx, int ny, int ns, bool allow_pipe,
                  int kmax = 1);
int heuristic_rows(int nx, int ny, int ns);
// Override, else cached tuning result, else heuristic (never tunes).
int current_rows(int kind, int model, int stencil, int scheme, int nx, int ny, int ns);
int tuned_rows(int kind, int model, int stencil, int scheme, int nx, int ny, int ns,
               hipStream_t s, const std::function<hipError_t(int)>& trial, int shape_key = 0,
               int fallback_ty = 0);
size_t align_up(size_t x, size_t a);
size_t field_bytes(const rd_problem* p);
int copy_state(double* const* dst, double* const* src, int nv, size_t bytes, hipStream_t s);

int workspace_jvp(const rd_problem* p, size_t* out);
// Workspace of rd_step_batched for probs[0 .. n-1] (validates each problem).
int batch_workspace(const rd_problem* probs, int32_t n, bool tangent, size_t* out);

// Optional finiteness check (rd_check.hip): extra workspace bytes while it is
// enabled (0 otherwise), and the scan itself (RD_OK when disabled).
size_t check_finite_bytes();
int check_finite_allowed(hipStream_t s);  // RD_EUNSUPPORTED inside a capture while enabled
int check_finite(double* const* f, int nf, size_t n, char* flag_ws, hipStream_t s, const char* what);

// 3-D stencils (rd_api_3d.cpp).
bool is_3d(int stencil);
size_t workspace_3d(const rd_problem* p, bool tangent);
int run_steps_3d(const rd_problem* p, const KConst& c, bool tangent, double* const* a, char* ws,
                 int64_t nsteps, double* checkpoints, int every, hipStream_t s);
size_t workspace_vjp_3d(const rd_problem* p);
int vjp_3d(const rd_problem* p, const KConst& c, const double* checkpoints, double* const* cot, char* ws,
           hipStream_t s);
int workspace_vjp(const rd_problem* p, size_t* out);
// Whether rd_vjp runs the fused reverse step (stage inputs recomputed in the
// adjoint kernel, halo 2 NS - 2 rows and columns) for this problem.
bool fused_adjoint(const rd_problem* p);

}  // namespace rd
