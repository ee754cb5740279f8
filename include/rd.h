/*
 * rd.h -- C ABI of librd.so, an MI355X (gfx950) library that advances 2-D
 * (and 3-D) cardiac reaction-diffusion systems
 *
 *     dz/dt = div(D grad z) + N[z],   z = (u, h1, h2, ...),
 *
 * in double precision with a fully explicit finite-difference time step.
 * The method is that of Marcotte & Grigoriev, "Implementation of PDE models
 * of cardiac dynamics on GPUs using OpenCL" (arXiv:1309.1720): Eq. (1) with
 * no-flux boundaries (Eq. 2) on an N x N Cartesian grid (Sect. 3), the
 * diffusion operator as a 5-point or 9-point stencil (Eq. 6) whose
 * out-of-domain points take the adjacent boundary value (Fig. 1), and
 * explicit Euler, Heun or classical fourth-order Runge-Kutta stages
 * (Sect. 3, Sect. 4).  The voltage u diffuses; FitzHugh-Nagumo's second
 * field v diffuses too (Eq. 3).
 *
 * Conventions shared by every entry point
 *   - Fields are FP64, one contiguous array per field ("structure of
 *     arrays"), row-major [ny][nx] ([nz][ny][nx] for the 3-D stencils) with x
 *     fastest, 8-byte aligned, on the current HIP device.  Cell (i, j) has
 *     centre ((i + 1/2) dx, (j + 1/2) dx).
 *   - Field order is the model's: Barkley (u, v); Fenton-Karma (u, v, w);
 *     Bueno-Orovio (u, v, w, s); FitzHugh-Nagumo (u, v); diffusion (u).
 *   - All field, tangent, cotangent, checkpoint and workspace pointers are
 *     DEVICE pointers owned by the caller.  rd_problem and its params array
 *     are HOST memory, read during the call only.
 *   - The library never allocates device memory.  Scratch space comes from
 *     the caller's workspace, whose size rd_workspace_bytes() reports.
 *   - Work is enqueued on `hip_stream` (a hipStream_t; NULL = the default
 *     stream) and the call returns without synchronising.  Argument errors
 *     are detected on the host before anything is enqueued; a device fault
 *     surfaces at the caller's next synchronisation.
 *   - Return value: RD_OK (0) or a negative rd_status.  rd_last_error()
 *     then returns a message for the calling thread.  No C++ exception
 *     crosses this interface.
 *   - Distinct pointers passed in one call must not alias.
 *   - The step entry points enqueue kernel launches and device-to-device
 *     copies only (no allocation, synchronisation or memset), so a HIP graph
 *     capture on `hip_stream` records them; replays repeat the call with the
 *     same pointers.  Inside a capture the autotuner does not time anything:
 *     make one call outside the capture first so the tuned plan is used.
 *     (The optional finiteness check of rd_set_check_finite synchronises and
 *     is refused inside a capture.)
 */
#ifndef RD_H
#define RD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RD_ABI_VERSION 2

/* Models (Sect. 2; the Barkley and Fenton-Karma models are additions). */
enum rd_model {
  RD_MODEL_DIFFUSION = 0,    /* N = 0, one field; a test model              */
  RD_MODEL_BARKLEY = 1,      /* 2 fields; params: a, b, eps                  */
  RD_MODEL_FENTON_KARMA = 2, /* 3 fields; params: tau_v+, tau_v1-, tau_v2-,
                                tau_w+, tau_w-, tau_d, tau_0, tau_r, tau_si,
                                k_si, u_c_si, u_c, u_v                       */
  RD_MODEL_BOCF = 3,         /* 4 fields (Eq. 5); params: u_o, u_u, theta_v,
                                theta_w, theta_v-, theta_o, tau_v1-, tau_v2-,
                                tau_v+, tau_w1-, tau_w2-, k_w-, u_w-, tau_w+,
                                tau_fi, tau_o1, tau_o2, tau_so1, tau_so2,
                                k_so, u_so, tau_s1, tau_s2, k_s, u_s, tau_si,
                                tau_w_inf, w_inf_star                        */
  RD_MODEL_FHN = 4           /* FitzHugh-Nagumo, Eq. (3): 2 fields, both
                                diffusive (v with delta D_par); params:
                                delta, eps, a1, a0                           */
};

/* Schemes (Sect. 3): explicit Euler (1 stage), Heun (2), classical RK4 (4);
 * and the first-order gate schemes the paper applies to the Bueno-Orovio
 * model (Table 1), for the gated models (Fenton-Karma, Bueno-Orovio) only:
 * the voltage takes an explicit Euler step and every gate g, whose rate is
 * alpha g + beta with alpha, beta frozen at z_n, takes
 *   Rush-Larsen:     g' = g e^{alpha dt} + (beta/alpha)(e^{alpha dt} - 1)
 *   implicit Euler:  g' = (g + dt beta) / (1 - dt alpha).
 * rd_step, rd_jvp, rd_vjp and rd_step_batched support them; other models
 * return RD_EUNSUPPORTED. */
enum rd_scheme {
  RD_SCHEME_EULER = 1,
  RD_SCHEME_HEUN = 2,
  RD_SCHEME_RK4 = 4,
  RD_SCHEME_RUSH_LARSEN = 5,
  RD_SCHEME_IMPLICIT_EULER = 6
};

/* Diffusion operators.
 *   RD_LAP5       D (W + E + N + S - 4C) / dx^2.
 *   RD_LAP9       Eq. (6): axial weight 2/3, diagonal weight 1/6, centre
 *                 balanced, times D / dx^2.
 *   RD_LAP9_ANISO div(D grad u) in conservative flux form for the tensor
 *                 D = D_perp I + (D_par - D_perp) f f^T, f = (cos t, sin t),
 *                 t linear in x from theta0 (x = 0) to theta1 (x = nx dx);
 *                 zero flux through the domain boundary.
 * 3-D operators on an nx x ny x nz grid (spacing dx in every direction; the
 * paper's conclusion anticipates 3-D tissue but prints no 3-D stencil).  The
 * 26 neighbours split into faces (6), edges (12) and corners (8); the operator
 * is D/dx^2 (w_f (faces - 6C) + w_e (edges - 12C) + w_c (corners - 8C)) with
 *   RD_LAP7   w = (1, 0, 0)           central differences
 *   RD_LAP19  w = (1/3, 1/6, 0)       isotropic leading error, no corners
 *   RD_LAP27  w = (7/15, 1/10, 1/30)  isotropic leading error, compact
 * Both isotropic members reduce to Eq. (6) on a single plane with mirrored
 * z-neighbours, as RD_LAP7 reduces to RD_LAP5.  Boundaries as in 2-D, in all
 * three directions.  rd_step and rd_jvp take them (every model and scheme),
 * rd_vjp too (every model and scheme), and rd_step_batched (each 3-D
 * instance's stage launches in turn). */
enum rd_stencil {
  RD_LAP5 = 5, RD_LAP9 = 9, RD_LAP9_ANISO = 10,
  RD_LAP7 = 7, RD_LAP19 = 19, RD_LAP27 = 27
};

/* Boundary conditions: no-flux (Eq. 2) via mirrored ghost cells (Fig. 1),
 * or periodic -- the alternative Sect. 3 describes, displacements that leave
 * the domain mapping to the opposite edge (in the flux form every face is
 * interior; the face between the last and the first column takes the tensor
 * at x = nx dx). */
enum rd_bc { RD_BC_NOFLUX = 0, RD_BC_PERIODIC = 1 };

/* Operations, for rd_workspace_bytes(): rd_step, rd_jvp, rd_vjp, and
 * rd_step_batched without (RD_OP_BATCHED) or with (RD_OP_BATCHED_JVP)
 * tangents. */
enum rd_op {
  RD_OP_STEP = 0, RD_OP_JVP = 1, RD_OP_VJP = 2, RD_OP_BATCHED = 3, RD_OP_BATCHED_JVP = 4
};

enum rd_status {
  RD_OK = 0,
  RD_EINVAL = -1,       /* invalid argument (null pointer, bad size, ...)     */
  RD_EUNSUPPORTED = -2, /* valid but unsupported combination                  */
  RD_EWORKSPACE = -3,   /* workspace missing or smaller than required         */
  RD_EHIP = -4,         /* HIP runtime error (message holds the HIP string)   */
  RD_ENONFINITE = -5    /* the result holds NaN or infinity (only while the
                           check of rd_set_check_finite is enabled)           */
};

/* One integration problem (the problem statement of Sect. 3). */
typedef struct rd_problem {
  uint32_t abi_version;   /* must equal RD_ABI_VERSION                        */
  int32_t model;          /* rd_model                                         */
  int32_t scheme;         /* rd_scheme                                        */
  int32_t stencil;        /* rd_stencil                                       */
  int32_t bc;             /* rd_bc                                            */
  int32_t nx, ny;         /* grid cells, each >= 1, nx * ny < 2^31            */
  double dx;              /* grid spacing (dy == dx), > 0                     */
  double dt;              /* time step, > 0                                   */
  int64_t nsteps;         /* steps to take, >= 0 (0 is a no-op)               */
  double D_par;           /* diffusivity (isotropic stencils use only this)   */
  double D_perp;          /* cross-fibre diffusivity, RD_LAP9_ANISO only      */
  double theta0, theta1;  /* fibre angle (radians), RD_LAP9_ANISO only        */
  double step_k;          /* sharpness k of the smoothed step H_k (Sect. 2),
                             > 0; +INFINITY selects the Heaviside step with
                             H(0) = 1                                         */
  const double* params;   /* host array of model parameters (order above)     */
  int32_t nparams;        /* its length; must match the model                 */
  int32_t checkpoint_every; /* rd_step: store the state every this many steps
                             into `checkpoints` (0 = none); rd_vjp: the
                             spacing of the checkpoints it is given            */
  int32_t nz;             /* planes: 1 for the 2-D stencils; >= 1 for the 3-D
                             ones, with nx * ny * nz < 2^40.  A 3-D field is
                             stored [nz][ny][nx], x fastest                   */
} rd_problem;

/* ABI version the library was built with (RD_ABI_VERSION). */
int rd_abi_version(void);

/* Number of fields of `model`, or RD_EINVAL. */
int rd_n_fields(int32_t model);

/* Number of parameters of `model`, or RD_EINVAL. */
int rd_n_params(int32_t model);

/* Number of checkpoint states rd_step writes for this problem:
 * ceil(nsteps / checkpoint_every), 0 when checkpoint_every == 0.
 * Checkpoint m is the state after m * checkpoint_every steps, stored as
 * [m][field][ny][nx] ([m][field][nz][ny][nx] in 3-D). */
int rd_checkpoint_count(const rd_problem* p, int64_t* out);

/* Bytes of device workspace an operation needs (the problem statement of
 * Sect. 3 fixes every size).
 *   RD_OP_STEP, RD_OP_JVP, RD_OP_VJP: for the one problem `p` (rd_step,
 *     rd_jvp, rd_vjp); *out is only written.
 *   RD_OP_BATCHED, RD_OP_BATCHED_JVP: for rd_step_batched on the batch
 *     p[0 .. nbatch-1] without / with tangents.  *out is read first: it must
 *     hold nbatch (1 <= nbatch <= 65536) on entry, and is overwritten with the
 *     byte count.  Every problem of the batch is validated.
 * The counts include the 256 bytes of the finiteness check while it is
 * enabled.  On error *out is left as it was. */
int rd_workspace_bytes(const rd_problem* p, int32_t op, size_t* out);

/*
 * rd_step -- advance the state by p->nsteps explicit steps, in place.
 *   fields       host array of n_fields device pointers; read as z(0),
 *                overwritten with z(nsteps).
 *   checkpoints  device array of rd_checkpoint_count(p) states, or NULL;
 *                receives z(m * checkpoint_every).
 *   ws, ws_bytes caller workspace, >= rd_workspace_bytes(p, RD_OP_STEP).
 * Each step is one fused kernel: every stage's stencil, reaction and
 * Euler-like update (Sect. 4) over an on-chip tile.
 */
int rd_step(const rd_problem* p, double* const* fields, double* checkpoints,
            void* ws, size_t ws_bytes, void* hip_stream);

/*
 * rd_step_noalloc -- rd_step for callers that cannot allocate device memory
 * or pass a workspace: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  Same arguments and results as rd_step
 * (bit for bit) without ws / ws_bytes: its scratch is a device array of
 * RD_NOALLOC_SCRATCH_BYTES the library owns, one per GPU, held until the
 * process ends.  It calls no hipMalloc / hipFree; the first call for a grid
 * shape may time candidate plans with HIP events, as rd_step does (not
 * during a capture).
 *   Problems whose rd_workspace_bytes(RD_OP_STEP) exceeds
 *   RD_NOALLOC_SCRATCH_BYTES fail with RD_EWORKSPACE (64 MiB: e.g. a
 *   2048^2 Barkley or a 1024^2 Fenton-Karma grid fits, a 2048^2
 *   Bueno-Orovio grid does not).
 *   All calls on one GPU share its array: calls that may overlap on one GPU
 *   (different streams, threads or processes' graphs replayed concurrently)
 *   race and must be ordered by the caller.  The array keeps the last call's
 *   contents; nothing in it needs to start at zero.
 */
#define RD_NOALLOC_SCRATCH_BYTES (64u << 20)
int rd_step_noalloc(const rd_problem* p, double* const* fields, double* checkpoints,
                    void* hip_stream);

/*
 * rd_jvp -- tangent-linear map of the finite-time flow (an addition to the
 * paper, motivated by its Newton-Krylov use case, Sect. 1).  Advances the
 * state z and a tangent dz together by p->nsteps steps, in place:
 *   fields    z(0) -> z(nsteps)
 *   tangents  dz(0) -> dPhi(z(0)) dz(0), the exact derivative of the
 *             discrete nsteps-step map.
 */
int rd_jvp(const rd_problem* p, double* const* fields, double* const* tangents,
           void* ws, size_t ws_bytes, void* hip_stream);

/*
 * rd_vjp -- adjoint of the finite-time flow (an addition to the paper).
 *   checkpoints  the states rd_step stored for the same problem (same
 *                nsteps and checkpoint_every > 0); only read.
 *   cotangents   host array of n_fields device pointers; read as
 *                lambda(nsteps), overwritten with
 *                lambda(0) = dPhi(z(0))^T lambda(nsteps).
 * States between checkpoints are recomputed into the workspace.
 * All stencils: the anisotropic flux form, which is not symmetric, is
 * transposed face by face (zero boundary flux and mirrored ghosts included).
 * The gate schemes transpose as the pointwise Jacobian of the step's
 * reaction and gate updates plus dt L^T on the voltage.
 */
int rd_vjp(const rd_problem* p, const double* checkpoints, double* const* cotangents,
           void* ws, size_t ws_bytes, void* hip_stream);

/*
 * rd_step_batched -- advance `nbatch` independent problems that differ only
 * in their grid sizes and time steps (model, scheme, stencil, boundary rule,
 * dx, nsteps, diffusivities, fibre angles and parameters agree;
 * RD_EUNSUPPORTED otherwise) in one launch per step over all of them (an
 * addition to the paper: ensembles, Krylov directions, and periodic orbits
 * whose periods T_i = nsteps dt_i differ); 3-D instances run their stage
 * launches one instance after another.
 *   fields[b]    host array of n_fields device pointers of problem b.
 *   tangents     NULL for a forward-only run, else tangents[b] as in
 *                rd_jvp: the tangents are advanced with the states.
 * Results equal per-problem rd_step / rd_jvp bit for bit.
 * rd_step_batched_workspace_bytes(probs, nbatch, with_tangents, out) is
 * rd_workspace_bytes(probs, with_tangents ? RD_OP_BATCHED_JVP :
 * RD_OP_BATCHED, out) with nbatch passed as an argument.
 */
int rd_step_batched_workspace_bytes(const rd_problem* probs, int32_t nbatch,
                                    int32_t with_tangents, size_t* out);
int rd_step_batched(const rd_problem* probs, int32_t nbatch, double* const* const* fields,
                    double* const* const* tangents, void* ws, size_t ws_bytes,
                    void* hip_stream);

/*
 * Krylov vector algebra (an addition to the paper: the matrix-free
 * Newton-Krylov solves on the time-T flow that Sect. 1 motivates, built on
 * rd_jvp / rd_step_batched).  A vector is a DEVICE array of n doubles (a
 * state's fields one after another); `x` is a HOST array of m device
 * pointers, each to n doubles.  Work is enqueued on `hip_stream`; sums run
 * in a fixed order (results do not depend on timing).
 *
 * rd_vec_gram:    out[k] = sum_i x[k][i] w[i], k < m, 1 <= m <= 64; `out` is
 *                 a device array of m doubles; workspace (device, 8-byte
 *                 aligned) of rd_vec_gram_workspace_bytes(m) bytes.
 * rd_vec_lincomb: y[i] = beta y[i] + sum_k coef[k] x[k][i], 0 <= m <= 64,
 *                 `coef` a HOST array of m doubles; y is not read when
 *                 beta == 0; y may be one of the x[k].
 */
int rd_vec_gram_workspace_bytes(int32_t m, size_t* out);
int rd_vec_gram(const double* const* x, int32_t m, const double* w, int64_t n, double* out,
                void* ws, size_t ws_bytes, void* hip_stream);
int rd_vec_lincomb(double* y, double beta, const double* const* x, const double* coef, int32_t m,
                   int64_t n, void* hip_stream);

/* Rows per wavefront band used by later calls from any thread (<= 0:
 * automatic choice).  A performance knob: results do not depend on it. */
int rd_set_tile_rows(int32_t rows);

/* Fixes the fused-step kernel variant for later calls: 0 = one wavefront
 * carrying every stage of a step, 1 = one wavefront per stage (stage-
 * pipelined workgroup); negative = chosen by the autotuner (default).  A
 * performance knob: both variants produce identical bits. */
int rd_set_kernel_variant(int32_t variant);

/* Kernel variant and band height the library uses for `op` (RD_OP_STEP or
 * RD_OP_JVP) on problem `p` (overrides, else the tuned choice, else the
 * heuristic starting plan). */
int rd_get_plan(const rd_problem* p, int32_t op, int32_t* variant, int32_t* rows);

/* Steps one launch of rd_step advances (temporal blocking, Sect. 4's kernel
 * fusion carried across steps): 1, 2, 4 or 8.  Only the models with cheap
 * reactions (diffusion, Barkley) chain steps, up to 8 stages per launch
 * (Euler 8 steps, Heun 4, RK4 2); launches never pass a checkpoint.
 * rd_set_steps_per_launch fixes it for later calls (capped by the model's
 * maximum; <= 0: chosen by the autotuner, the default); other values return
 * RD_EINVAL.  A performance knob: results do not depend on it.
 * rd_get_steps_per_launch reports the value rd_step uses for `p`. */
int rd_set_steps_per_launch(int32_t steps);
int rd_get_steps_per_launch(const rd_problem* p, int32_t* steps);

/* Band height the library uses for `op` (RD_OP_STEP, RD_OP_JVP, RD_OP_VJP) on
 * problem `p`: the override, else the autotuner's cached choice, else its
 * heuristic starting value.  For RD_OP_VJP, the band height of the reverse
 * step's adjoint kernel (the fused one where rd_vjp runs it). */
int rd_get_tile_rows(const rd_problem* p, int32_t op, int32_t* rows);

/* Enables (non-zero, the default) or disables the band-height autotuner.
 * When enabled, the first call for each (operation, model, stencil, scheme,
 * nx, ny) times candidate band heights with HIP events on the caller's stream
 * (trial launches read the inputs and write only workspace) and blocks until
 * those timings finish; later calls reuse the choice.  Never inside a stream
 * capture.  Results do not depend on it. */
int rd_set_autotune(int32_t enable);

/* Reverse step of rd_vjp for the models with at most two fields (diffusion,
 * Barkley, FitzHugh-Nagumo) under Heun or RK4 with no-flux boundaries:
 * non-zero (the default) recomputes each step's stage inputs inside the
 * adjoint kernel, 0 writes them to the workspace with a separate sweep first
 * (the path every other model and scheme takes).  Results are bit-identical;
 * the first moves fewer bytes. */
int rd_set_fused_adjoint(int32_t enable);

/* Enables (non-zero) or disables (0, the default) a debugging check: after
 * rd_step, rd_jvp, rd_vjp and rd_step_batched have enqueued their work, a
 * small kernel scans the fields they produced and the call returns
 * RD_ENONFINITE if any value is NaN or infinite.  While enabled, every call
 * synchronises its stream (so it cannot be captured in a HIP graph; calls
 * inside a capture return RD_EUNSUPPORTED) and needs 256 more workspace bytes,
 * which rd_workspace_bytes and rd_step_batched_workspace_bytes then include. */
int rd_set_check_finite(int32_t enable);

/* Message for the last failed call on this thread ("" if none). */
const char* rd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RD_H */
