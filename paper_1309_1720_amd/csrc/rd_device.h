// rd_device.h -- device-side building blocks of the explicit reaction-diffusion
// step (Marcotte & Grigoriev, arXiv:1309.1720): kernel constants, the smoothed
// step H_k (Sect. 2), the reaction terms N[z] of Eq. (1), their pointwise
// Jacobians, and the diffusion operators (Eq. 6 and the anisotropic flux form)
// evaluated across a wavefront whose 64 lanes hold 64 consecutive columns.
//
// All arithmetic is FP64.  Sources are built with -ffp-contract=off so that
// every product and sum rounds where the source writes it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rd.h"

namespace rd {

constexpr int kMaxFields = 4;
constexpr int kWave = 64;
constexpr double kAlphaAxial = 2.0 / 3.0;  // Eq. (6) axial weight
constexpr double kAlphaDiag = 1.0 / 6.0;   // Eq. (6) diagonal weight

// Model constants, derived on the host from the caller's parameters.  Constant
// divisors are stored as reciprocals; u-dependent time constants are divided.
struct BarkleyC { double b, inv_a, inv_eps; };
struct FhnC { double eps, a1, a0; };
// (1 + tanh(k (u - u_x))) / 2 is evaluated as 1 / (1 + e^(a u + b)) with
// a = -2k, b = 2k u_x (lg_*); tau(u) blends as tau_1 + h (tau_2 - tau_1).
struct FentonKarmaC {
  double u_c, u_v, inv_tau_d, inv_tau_0, inv_tau_r, inv_tau_si, lg_a, lg_b,
      tau_v2m, dtau_vm, inv_tau_vp, inv_tau_wm, inv_tau_wp;
};
// tau_w^- and tau_so blend through logistics and keep both ends; the other
// tau(u) blend as tau_1 + H (tau_2 - tau_1).
struct BocfC {
  double u_o, u_u, th_v, th_w, th_vm, th_o, tau_v1m, dtau_vm, inv_tau_vp, tau_w1m,
      tau_w2m, lg_wm_a, lg_wm_b, inv_tau_wp, inv_tau_fi, tau_o1, dtau_o, tau_so1, tau_so2,
      lg_so_a, lg_so_b, tau_s1, dtau_s, lg_s_a, lg_s_b, inv_tau_si, inv_tau_winf, w_infstar;
};
union ModelC {
  BarkleyC bk;
  FhnC fh;
  FentonKarmaC fk;
  BocfC bo;
  double raw[32];
};

// Everything a step kernel needs besides field pointers (passed by value).
struct KConst {
  int nx, ny;        // grid
  int nsx, nby, ty;  // launch geometry: column strips, row bands, rows per band
  int sharp;         // 1: Heaviside step instead of H_k
  int variant;       // fused-step kernel variant (StepVariant)
  int ksteps;        // steps per launch of the state-only sweep (1, 2, 4, 8)
  int periodic;      // 1: periodic boundaries (RD_BC_PERIODIC), 0: no-flux
  double k;          // H_k sharpness (+inf for the Heaviside step)
  double k6;         // dH_k/dt scale 6 k (0 for the Heaviside step)
  double dt, h2, h6; // dt, dt/2, dt/6
  // Scale of the diffusion operator of diffusive field d (u, then v for
  // FitzHugh-Nagumo, whose v diffuses delta times faster): (D_par rel_d) / dx^2
  // for the isotropic stencils, rel_d / dx^2 for the anisotropic flux form.
  double dcoef[2];
  double theta0, dtheta, n_total, d_perp, dd;  // fibre field, dd = D_par - D_perp
  ModelC m;
};

// NV fields per cell; the first NDIFF of them diffuse.  GATED models have
// gating variables (fields NDIFF .. NV-1) whose rates are affine in the gate
// itself, dg/dt = alpha g + beta (Reaction<>::gates gives alpha and beta).
template <int MODEL> struct ModelTraits;
template <> struct ModelTraits<RD_MODEL_DIFFUSION> { static constexpr int NV = 1, NDIFF = 1; static constexpr bool GATED = false; };
template <> struct ModelTraits<RD_MODEL_BARKLEY> { static constexpr int NV = 2, NDIFF = 1; static constexpr bool GATED = false; };
template <> struct ModelTraits<RD_MODEL_FENTON_KARMA> { static constexpr int NV = 3, NDIFF = 1; static constexpr bool GATED = true; };
template <> struct ModelTraits<RD_MODEL_BOCF> { static constexpr int NV = 4, NDIFF = 1; static constexpr bool GATED = true; };
template <> struct ModelTraits<RD_MODEL_FHN> { static constexpr int NV = 2, NDIFF = 2; static constexpr bool GATED = false; };

// ---------------------------------------------------------------------------
// Smoothed step: t = kx + 1/2 clamped to [0, 1], H = t^2 (3 - 2t).  Clamping
// reproduces the 0 and 1 branches exactly (0*0*3 = 0, 1*1*1 = 1).  The
// Heaviside limit uses the same instructions with k = +inf: t is -inf or +inf
// away from x = 0 and NaN at x = 0 (inf * 0), and the clamp max(min(t, 1), 0)
// takes NaN to 1 (min returns its non-NaN operand), so H(0) = 1 -- no branch
// and no select.  Used only by the gated models, so it may fuse multiply-adds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double step_h(double x, const KConst& c) {
  double t = fma(c.k, x, 0.5);
  t = fmax(fmin(t, 1.0), 0.0);
  return (t * t) * fma(-2.0, t, 3.0);
}

// H and dH/dx = 6 k t (1 - t), which is zero outside the transition and for
// the Heaviside step (k6 = 0 there, and t (1 - t) = 0).
__device__ __forceinline__ void step_h_d(double x, const KConst& c, double& h, double& dh) {
  double t = fma(c.k, x, 0.5);
  t = fmax(fmin(t, 1.0), 0.0);
  h = (t * t) * fma(-2.0, t, 3.0);
  dh = c.k6 * (t * (1.0 - t));
}

// ---------------------------------------------------------------------------
// Forward-mode dual numbers: a value and one directional derivative.  The
// reaction code is written once over a scalar type T; instantiated with Dual
// it returns N(y) and J_N(y) dy together.  Each operation computes its value
// exactly as the double version does, so the value parts are bit-identical
// to a plain evaluation.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() = default;
  __host__ __device__ explicit constexpr Dual(double x) : v(x), d(0.0) {}
  __host__ __device__ constexpr Dual(double x, double dx) : v(x), d(dx) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
__device__ __forceinline__ Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
__device__ __forceinline__ Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
__device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ Dual operator/(double a, Dual b) {
  const double q = a / b.v;
  return Dual(q, -(q * b.d) / b.v);
}
__device__ __forceinline__ Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
// ---------------------------------------------------------------------------
// Lean FP64 elementary functions for the reaction terms.
//
// exp: Cody-Waite argument reduction x = n ln2 + r, |r| <= ln2/2, with ln2
// split into a high part whose product with n is exact and a low part, then
// e^r ~ 1 + r + r^2/2 + r^3 h(r) with h of degree 8, its coefficients the
// minimax fit of the relative error on |r| <= ln2/2 by the Remez exchange
// algorithm (exp_poly_fit.py beside this file; approximation error 2.4e-17,
// the low-order coefficients 1, 1, 1/2 kept exact so that they are inline
// operands), by Horner's rule in fused multiply-adds, scaled by 2^n.  The
// polynomial evaluates within 0.6 ulp in double; about 2 ulp in all; 18 FP64
// operations against ~40 for the general library routine.
//
// recip: the hardware reciprocal estimate (relative error below 3e-8)
// refined by one third-order step: with e = 1 - d r, 1/d = r / (1 - e) =
// r (1 + e + e^2 + ...), so r + r (e + e^2) leaves a truncation of order e^3
// (below 1e-22) and only the three fused multiply-adds' rounding: as accurate
// as two Newton-Raphson steps r <- r + r e (within 1 ulp, in practice
// correctly rounded, for the positive, finite, normal divisors the reactions
// use: time constants, 1 + exp(.)), one multiply-add cheaper.
// ---------------------------------------------------------------------------
// e^x for x in [-1e4, 1e4] (n stays in int range; exp saturates far earlier).
__device__ __forceinline__ double exp_core(double x) {
  const double n = __builtin_rint(x * 1.4426950408889634);   // log2(e)
  double r = fma(-n, 6.93147180369123816490e-01, x);        // ln2 high part (exact product)
  r = fma(-n, 1.90821492927058770002e-10, r);                // ln2 low part
  double p = 2.2976443849446772e-08;  // r^11 ... r^3: the minimax coefficients
  p = fma(p, r, 2.7622226153978235e-07);
  p = fma(p, r, 2.7563857293242605e-06);
  p = fma(p, r, 2.4801516346798477e-05);
  p = fma(p, r, 1.9841262673010967e-04);
  p = fma(p, r, 1.3888888920512005e-03);
  p = fma(p, r, 8.3333333365280360e-03);
  p = fma(p, r, 4.1666666666619970e-02);
  p = fma(p, r, 1.6666666666661958e-01);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return __builtin_amdgcn_ldexp(p, (int)n);
}

__device__ __forceinline__ double exp_lean(double x) { return exp_core(fmin(fmax(x, -1.0e4), 1.0e4)); }

__device__ __forceinline__ double recip(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  const double e = fma(-d, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// e^x - 1 without the cancellation of exp(x) - 1 near 0: for |x| <= ln2/2
// the Taylor series x (1 + x/2! + ... + x^13/14!) (truncation < 1e-17
// relative), elsewhere exp(x) - 1 (no cancellation there).  Both are
// evaluated and one selected.
__device__ __forceinline__ double expm1_lean(double x) {
  double q = 1.0 / 87178291200.0;  // 1/14!
  q = fma(q, x, 1.0 / 6227020800.0);
  q = fma(q, x, 1.0 / 479001600.0);
  q = fma(q, x, 1.0 / 39916800.0);
  q = fma(q, x, 1.0 / 3628800.0);
  q = fma(q, x, 1.0 / 362880.0);
  q = fma(q, x, 1.0 / 40320.0);
  q = fma(q, x, 1.0 / 5040.0);
  q = fma(q, x, 1.0 / 720.0);
  q = fma(q, x, 1.0 / 120.0);
  q = fma(q, x, 1.0 / 24.0);
  q = fma(q, x, 1.0 / 6.0);
  q = fma(q, x, 0.5);
  q = fma(q, x, 1.0);
  const double small = x * q;
  const double large = exp_lean(x) - 1.0;
  return fabs(x) <= 0.34657359027997264 ? small : large;
}

__device__ __forceinline__ double exp(double a) { return exp_lean(a); }
__device__ __forceinline__ double expm1(double a) { return expm1_lean(a); }
__device__ __forceinline__ Dual exp(Dual a) {
  const double e = exp_lean(a.v);
  return Dual(e, e * a.d);
}
__device__ __forceinline__ Dual expm1(Dual a) {
  return Dual(expm1_lean(a.v), exp_lean(a.v) * a.d);
}
__device__ __forceinline__ Dual recip(Dual a) {
  const double r = recip(a.v);
  return Dual(r, -(r * a.d) * r);
}

// mad(a, b, c) = a b + c with one rounding (value part identical for double
// and Dual).
__device__ __forceinline__ double mad(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ Dual mad(Dual a, double b, Dual c) {
  return Dual(fma(a.v, b, c.v), fma(a.d, b, c.d));
}
__device__ __forceinline__ Dual mad(double a, Dual b, Dual c) {
  return Dual(fma(a, b.v, c.v), fma(a, b.d, c.d));
}
__device__ __forceinline__ Dual mad(Dual a, double b, double c) {
  return Dual(fma(a.v, b, c), a.d * b);
}
__device__ __forceinline__ Dual mad(Dual a, Dual b, Dual c) {
  return Dual(fma(a.v, b.v, c.v), fma(a.d, b.v, fma(a.v, b.d, c.d)));
}
__device__ __forceinline__ Dual step_h(Dual x, const KConst& c) {
  double h, dh;
  step_h_d(x.v, c, h, dh);
  return Dual(h, dh * x.d);
}

// How a reaction evaluates H_k.  kHkAny: the instructions of step_h, right for
// a finite k and for the Heaviside limit alike.  kHkSmooth (finite k only):
// the pairs H(x), H(-x) share one evaluation, since t(-x) = 1 - t(x) and
// H(1 - t) = 1 - H(t).  kHkSharp (k = inf only): the Heaviside function,
// H(x) = 1 for x >= 0 (so H(0) = H(-0) = 1, and the pairs do not complement).
// The fused step kernels pick kHkSmooth or kHkSharp per call; both give the
// function kHkAny gives, to rounding (kHkSharp exactly).
enum HkEval { kHkAny = 0, kHkSmooth = 1, kHkSharp = 2 };

// kHkSmooth: t = kx + 1/2 is finite, so its clamp to [0, 1] is written
// max-then-min, which the compiler folds into the clamp bit of the
// multiply-add that forms t (no separate min/max instructions).
__device__ __forceinline__ double step_t_smooth(double x, const KConst& c) {
  return fmin(fmax(fma(c.k, x, 0.5), 0.0), 1.0);
}
template <int HK>
__device__ __forceinline__ double hk(double x, const KConst& c) {
  if constexpr (HK == kHkSharp) {
    return x >= 0.0 ? 1.0 : 0.0;
  } else if constexpr (HK == kHkSmooth) {
    const double t = step_t_smooth(x, c);
    return (t * t) * fma(-2.0, t, 3.0);
  } else {
    return step_h(x, c);
  }
}
template <int HK>
__device__ __forceinline__ Dual hk(Dual x, const KConst& c) {
  if constexpr (HK == kHkSharp) {
    return Dual(x.v >= 0.0 ? 1.0 : 0.0, 0.0);
  } else if constexpr (HK == kHkSmooth) {
    const double t = step_t_smooth(x.v, c);
    return Dual((t * t) * fma(-2.0, t, 3.0), (c.k6 * (t * (1.0 - t))) * x.d);
  } else {
    return step_h(x, c);
  }
}
// h = H(x), hn = H(-x).  -x is exact, so kHkAny and kHkSharp evaluate
// H(th - u) exactly as written when x = u - th.
template <int HK, class T>
__device__ __forceinline__ void hk_pair(T x, const KConst& c, T& h, T& hn) {
  h = hk<HK>(x, c);
  if constexpr (HK == kHkSmooth) hn = 1.0 - h;
  else hn = hk<HK>(-x, c);
}

// (1 + tanh(x)) / 2 written as the logistic function 1 / (1 + exp(-2x)): the
// same function, evaluated with one exp and one division (an FP64 tanh costs
// several times more), and without the cancellation 1 + tanh(x) suffers for
// x << 0.  The caller passes the exponent e = -2x, formed from u by one
// multiply-add with host-computed constants.
//
// The exponent is clamped to [-1e4, 600] first (the clamp of exp_lean, with a
// lower upper end).  Beyond 600 the logistic is below 3e-261 (and
// (1 + tanh x)/2 rounds to exactly 0 in double), but exp(e) would overflow to
// +inf from e = 709.8 on, and the reciprocal's Newton step turns 1/inf into
// inf * 0 = NaN; 600 also leaves tau e^e finite for time constants tau up to
// 1e47 (logistic_blend_recip).  Clamped, the value stays a positive double
// below 3e-261 and its derivative is 0, as is the derivative of the rounded
// (1 + tanh x)/2 there.  Reached only far outside the physiological range
// (Fenton-Karma u < -30, Bueno-Orovio u < -4.6).
constexpr double kExpCap = 600.0;
__device__ __forceinline__ double exp_capped(double e) { return exp_core(fmax(fmin(e, kExpCap), -1.0e4)); }
__device__ __forceinline__ Dual exp_capped(Dual e) {
  const double x = exp_capped(e.v);
  return Dual(x, e.v > kExpCap ? 0.0 : x * e.d);
}
template <class T>
__device__ __forceinline__ T logistic_of_exponent(T e) {
  return recip(1.0 + exp_capped(e));
}
// 1 / (tau1 + (tau2 - tau1) L) with L = 1 / (1 + E), E = e^e, the logistic
// above: equal to (1 + E) / (tau1 E + tau2), one reciprocal instead of two.
template <class T>
__device__ __forceinline__ T logistic_blend_recip(T e, double tau1, double tau2) {
  const T E = exp_capped(e);
  return (1.0 + E) * recip(mad(E, tau1, tau2));
}

// ---------------------------------------------------------------------------
// Reaction rates f = N(y).  Barkley rounds every operation as written (and so
// matches the oracle bit for bit); the gated models fuse multiply-adds and
// multiply by reciprocals of their u-dependent time constants.  HK selects
// the evaluation of H_k (HkEval); models without H_k ignore it.
// ---------------------------------------------------------------------------
template <int MODEL> struct Reaction;

template <> struct Reaction<RD_MODEL_DIFFUSION> {
  template <class T, int HK = kHkAny>
  __device__ __forceinline__ static void rates(const KConst&, const T*, T* f) {
    f[0] = T(0.0);
  }
};

// Barkley: du = (1/eps) u (1 - u)(u - (v + b)/a), dv = u - v.
template <> struct Reaction<RD_MODEL_BARKLEY> {
  template <class T, int HK = kHkAny>
  __device__ __forceinline__ static void rates(const KConst& c, const T* y, T* f) {
    const BarkleyC& m = c.m.bk;
    const T u = y[0], v = y[1];
    const T uth = (v + m.b) * m.inv_a;
    f[0] = ((m.inv_eps * u) * (1.0 - u)) * (u - uth);
    f[1] = u - v;
  }
};

// FitzHugh-Nagumo, Eq. (3) without its diffusion terms:
// du = u - v - u^3, dv = eps (u - a1 v - a0).  Rounded as written (matches the
// oracle bit for bit).
template <> struct Reaction<RD_MODEL_FHN> {
  template <class T, int HK = kHkAny>
  __device__ __forceinline__ static void rates(const KConst& c, const T* y, T* f) {
    const FhnC& m = c.m.fh;
    const T u = y[0], v = y[1];
    f[0] = (u - v) - (u * u) * u;
    f[1] = m.eps * ((u - m.a1 * v) - m.a0);
  }
};

// Fenton-Karma three-variable model, gates through H_k:
// J_fi = -v p (1-u)(u-u_c)/tau_d, J_so = u(1-p)/tau_0 + p/tau_r,
// J_si = -w (1 + tanh(k_si (u - u_csi))) / (2 tau_si),
// dv = (1-p)(1-v)/tau_v^-(u) - p v/tau_v^+, dw = (1-p)(1-w)/tau_w^- - p w/tau_w^+.
template <> struct Reaction<RD_MODEL_FENTON_KARMA> {
  template <class T, int HK = kHkAny>
  __device__ __forceinline__ static void rates(const KConst& c, const T* y, T* f) {
    const FentonKarmaC& m = c.m.fk;
    const T u = y[0], v = y[1], w = y[2];
    const T p = hk<HK>(u - m.u_c, c);
    const T q = hk<HK>(u - m.u_v, c);
    const T one_p = 1.0 - p;
    const T j_fi = -(((v * p) * (1.0 - u)) * (u - m.u_c)) * m.inv_tau_d;
    const T j_so = mad(u * one_p, m.inv_tau_0, p * m.inv_tau_r);
    const T j_si = -(w * logistic_of_exponent(mad(u, m.lg_a, m.lg_b))) * m.inv_tau_si;
    const T tau_vm = mad(q, m.dtau_vm, T(m.tau_v2m));
    f[0] = -((j_fi + j_so) + j_si);
    f[1] = mad(-(p * v), m.inv_tau_vp, (one_p * (1.0 - v)) * recip(tau_vm));
    f[2] = mad(one_p * (1.0 - w), m.inv_tau_wm, -(p * w) * m.inv_tau_wp);
  }
  // dv = alpha_v v + beta_v, dw = alpha_w w + beta_w (the same rates, sorted
  // by powers of the gate).
  template <class T, int HK = kHkAny>
  __device__ __forceinline__ static void gates(const KConst& c, const T* y, T* al, T* be) {
    const FentonKarmaC& m = c.m.fk;
    const T u = y[0];
    const T p = hk<HK>(u - m.u_c, c);
    const T q = hk<HK>(u - m.u_v, c);
    const T one_p = 1.0 - p;
    const T r_vm = recip(mad(q, m.dtau_vm, T(m.tau_v2m)));
    al[1] = -(one_p * r_vm) - p * m.inv_tau_vp;
    be[1] = one_p * r_vm;
    al[2] = -(one_p * m.inv_tau_wm) - p * m.inv_tau_wp;
    be[2] = one_p * m.inv_tau_wm;
  }
};

// Bueno-Orovio four-variable model, Eq. (5) with the currents and the
// alpha/beta gate form; tau(u), v_inf, w_inf as in Bueno-Orovio et al. (2008).
// The u-dependent quantities both the rates and the gate coefficients use.
template <class T>
struct BocfTerms {
  T h_v, h_v_neg, h_w, h_w_neg, h_o, v_inf;
  T r_vm, r_wm, r_s;  // 1/tau_v^-, 1/tau_w^-, 1/tau_s
  T w_inf, s_inf;
};
template <> struct Reaction<RD_MODEL_BOCF> {
  template <class T, int HK>
  __device__ __forceinline__ static BocfTerms<T> terms(const KConst& c, const T& u) {
    const BocfC& m = c.m.bo;
    BocfTerms<T> t;
    hk_pair<HK>(u - m.th_v, c, t.h_v, t.h_v_neg);
    hk_pair<HK>(u - m.th_w, c, t.h_w, t.h_w_neg);
    T h_vm;
    hk_pair<HK>(u - m.th_vm, c, h_vm, t.v_inf);  // v_inf = H(th_v^- - u)
    t.h_o = hk<HK>(u - m.th_o, c);
    // 1/tau_v^- and 1/tau_w^- (tau_w^- = (E tau_w1^- + tau_w2^-) / (1 + E), the
    // logistic blend) from one reciprocal of the product of the two
    // denominators; each product holds at most one exponential (capped), so it
    // stays finite.  One FP64 reciprocal costs about as much as four FMAs.
    {
      const T E_wm = exp_capped(mad(u, m.lg_wm_a, m.lg_wm_b));
      const T d_wm = mad(E_wm, m.tau_w1m, T(m.tau_w2m));
      const T t_vm = mad(h_vm, m.dtau_vm, T(m.tau_v1m));
      const T R = recip(t_vm * d_wm);
      t.r_vm = R * d_wm;
      t.r_wm = (1.0 + E_wm) * (t_vm * R);
    }
    t.r_s = recip(mad(t.h_w, m.dtau_s, T(m.tau_s1)));                  // tau_s1 + H (tau_s2 - tau_s1)
    // w_inf = (1 - H_o)(1 - u / tau_winf) + H_o w_inf*
    const T a = mad(-u, m.inv_tau_winf, 1.0);
    t.w_inf = mad(t.h_o, m.w_infstar - a, a);
    t.s_inf = logistic_of_exponent(mad(u, m.lg_s_a, m.lg_s_b));
    return t;
  }

  // dv, dw as alpha g + beta (as the rates below form them); ds = (s_inf - s)/tau_s
  // gives alpha_s = -1/tau_s, beta_s = s_inf/tau_s.
  template <class T, int HK = kHkAny>
  __device__ __forceinline__ static void gates(const KConst& c, const T* y, T* al, T* be) {
    const BocfC& m = c.m.bo;
    const BocfTerms<T> t = terms<T, HK>(c, y[0]);
    al[1] = mad(-t.h_v, m.inv_tau_vp, -(t.h_v_neg * t.r_vm));
    be[1] = (t.h_v_neg * t.v_inf) * t.r_vm;
    al[2] = mad(-t.h_w, m.inv_tau_wp, -(t.h_w_neg * t.r_wm));
    be[2] = (t.h_w_neg * t.w_inf) * t.r_wm;
    al[3] = -t.r_s;
    be[3] = t.s_inf * t.r_s;
  }

  template <class T, int HK = kHkAny>
  __device__ __forceinline__ static void rates(const KConst& c, const T* y, T* f) {
    const BocfC& m = c.m.bo;
    const T u = y[0], v = y[1], w = y[2], s = y[3];
    const BocfTerms<T> t = terms<T, HK>(c, u);
    // 1/tau_so (logistic blend) and 1/tau_o from one reciprocal, as above.
    const T E_so = exp_capped(mad(u, m.lg_so_a, m.lg_so_b));
    const T d_so = mad(E_so, m.tau_so1, T(m.tau_so2));
    const T t_o = mad(t.h_o, m.dtau_o, T(m.tau_o1));
    const T R = recip(t_o * d_so);
    const T r_so = (1.0 + E_so) * (t_o * R);
    const T r_o = R * d_so;
    const T j_fi = -(((v * t.h_v) * (u - m.th_v)) * (m.u_u - u)) * m.inv_tau_fi;
    const T j_so = mad((u - m.u_o) * t.h_w_neg, r_o, t.h_w * r_so);
    const T j_si = -((t.h_w * w) * s) * m.inv_tau_si;
    f[0] = -((j_fi + j_so) + j_si);
    const T alpha_v = mad(-t.h_v, m.inv_tau_vp, -(t.h_v_neg * t.r_vm));
    const T beta_v = (t.h_v_neg * t.v_inf) * t.r_vm;
    f[1] = mad(alpha_v, v, beta_v);
    const T alpha_w = mad(-t.h_w, m.inv_tau_wp, -(t.h_w_neg * t.r_wm));
    const T beta_w = (t.h_w_neg * t.w_inf) * t.r_wm;
    f[2] = mad(alpha_w, w, beta_w);
    // (s_inf - s) / tau_s with s_inf = 1 / (1 + E) written as
    // (1 - s (1 + E)) / ((1 + E) tau_s): one reciprocal instead of two.
    const T one_e = 1.0 + exp_capped(mad(u, m.lg_s_a, m.lg_s_b));
    f[3] = mad(-s, one_e, T(1.0)) * recip(one_e * mad(t.h_w, m.dtau_s, T(m.tau_s1)));
  }
};

// One step of the gate schemes for a gate g with rate alpha g + beta frozen
// over the step: GATE = 1 Rush-Larsen (exact for the frozen linear equation),
// GATE = 2 implicit Euler.
template <int GATE, class T>
__device__ __forceinline__ T gate_step(T g, T al, T be, double dt) {
  if constexpr (GATE == 1) {
    const T x = al * dt;
    return g * exp(x) + (be / al) * expm1(x);
  } else {
    return (g + dt * be) / (1.0 - dt * al);
  }
}

// The step of a gate scheme on a packed row y (state, then tangent when TAN):
// explicit Euler for the diffusive field with its full rate k (diffusion +
// reaction), gate_step for the gates.  zn receives the new packed row.
template <int MODEL, bool TAN, int GATE, int HK = kHkAny>
__device__ __forceinline__ void gate_scheme_step(const KConst& c, const double* y, const double* k,
                                                 double* zn) {
  constexpr int NV = ModelTraits<MODEL>::NV;
  static_assert(ModelTraits<MODEL>::GATED && ModelTraits<MODEL>::NDIFF == 1, "gated models only");
  zn[0] = y[0] + c.dt * k[0];
  if constexpr (!TAN) {
    double al[NV], be[NV];
    Reaction<MODEL>::template gates<double, HK>(c, y, al, be);
#pragma unroll
    for (int g = 1; g < NV; ++g) zn[g] = gate_step<GATE>(y[g], al[g], be[g], c.dt);
  } else {
    zn[NV] = y[NV] + c.dt * k[NV];
    Dual yd[NV], al[NV], be[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) yd[f] = Dual(y[f], y[NV + f]);
    Reaction<MODEL>::template gates<Dual, HK>(c, yd, al, be);
#pragma unroll
    for (int g = 1; g < NV; ++g) {
      const Dual r = gate_step<GATE>(yd[g], al[g], be[g], c.dt);
      zn[g] = r.v;
      zn[NV + g] = r.d;
    }
  }
}

// N(y) (TAN = false) or N(y) and J_N(y) dy (TAN = true) for a packed row
// y[0..NV) = state, y[NV..2NV) = tangent; results packed the same way.
template <int MODEL, bool TAN, int HK = kHkAny>
__device__ __forceinline__ void eval_rates(const KConst& c, const double* y, double* k) {
  constexpr int NV = ModelTraits<MODEL>::NV;
  if constexpr (!TAN) {
    Reaction<MODEL>::template rates<double, HK>(c, y, k);
  } else {
    Dual yd[NV], kd[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) yd[f] = Dual(y[f], y[NV + f]);
    Reaction<MODEL>::template rates<Dual, HK>(c, yd, kd);
#pragma unroll
    for (int f = 0; f < NV; ++f) {
      k[f] = kd[f].v;
      k[NV + f] = kd[f].d;
    }
  }
}

// ---------------------------------------------------------------------------
// Cross-lane access.  Lane l holds column x0 + l; the previous/next lane holds
// the west/east neighbour.  Lanes 0 and 63 are halo lanes whose results never
// reach an output.
// ---------------------------------------------------------------------------
// The moves are DPP whole-wavefront shifts by one lane (wave_shr:1 reads the
// lane below, wave_shl:1 the lane above), executed by the vector ALU.  Lanes
// 0 and 63, which have no source lane, read zero; they are halo lanes.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = (int)b, hi = (int)(b >> 32);
  const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, true);
  const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((long long)hi2 << 32) | (unsigned int)lo2);
}
__device__ __forceinline__ double from_west(double v) { return dpp_shift<kDppWaveShr1>(v); }
__device__ __forceinline__ double from_east(double v) { return dpp_shift<kDppWaveShl1>(v); }

// Per-lane geometry of a column.
struct Column {
  int gx;        // global column of this lane (may lie outside [0, nx))
  bool west;     // gx <= 0: west neighbour is the mirror ghost (this column)
  bool east;     // gx >= nx-1: east neighbour is the mirror ghost
  double dxx_e, dxy_e4, dxy_c4, dyy_c;  // anisotropic tensor at face gx+1/2 / centre gx
  double dxx_w, dxy_w4;                 // ... at face gx-1/2, as the west neighbour computes it
};

// Whether the 64 columns of the strip starting at column x0 include the first
// or the last column of the grid (wave-uniform); periodic grids have no edge.
__device__ __forceinline__ bool strip_touches_edge(int x0, const KConst& c) {
  return !c.periodic && (x0 <= 0 || x0 + kWave - 1 >= c.nx - 1);
}

// x mod n in [0, n) for any int x (periodic indices).
__device__ __forceinline__ int wrap_index(int x, int n) {
  const int r = x % n;
  return r < 0 ? r + n : r;
}

// The array index of column/row x: clamped into the grid for no-flux
// boundaries (those values are mirrored or unused), wrapped for periodic ones.
__device__ __forceinline__ int grid_index(int x, int n, const KConst& c) {
  return c.periodic ? wrap_index(x, n) : min(max(x, 0), n - 1);
}

// Launch order -> work order.  Workgroups are handed to the eight XCDs
// round-robin (workgroup b runs on XCD b mod 8), and each XCD has its own L2.
// This bijection of [0, nblocks) numbers the workgroups of one XCD
// consecutively, so that work items with adjacent numbers -- vertically
// adjacent bands of one strip, which share halo rows -- meet in the same L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_order(int b, int nblocks) {
  const int q = nblocks / kXcds, rem = nblocks % kXcds;
  const int x = b % kXcds;
  return x * q + min(x, rem) + b / kXcds;
}

__device__ __forceinline__ Column make_column(int gx, const KConst& c, bool aniso) {
  Column col;
  col.gx = gx;
  col.west = !c.periodic && gx <= 0;
  col.east = !c.periodic && gx >= c.nx - 1;
  col.dxx_e = col.dxy_e4 = col.dxy_c4 = col.dyy_c = col.dxx_w = col.dxy_w4 = 0.0;
  if (aniso) {
    // periodic: the tensor of the wrapped column (the face east of the last
    // column lies at x = nx dx, as does the face west of the first)
    const double g = c.periodic ? (double)wrap_index(gx, c.nx) : (double)gx;
    const double gw = c.periodic ? (double)wrap_index(gx - 1, c.nx) : (double)(gx - 1);
    const double th_f = c.theta0 + c.dtheta * ((g + 1.0) / c.n_total);
    const double th_w = c.theta0 + c.dtheta * ((gw + 1.0) / c.n_total);
    const double th_c = c.theta0 + c.dtheta * ((g + 0.5) / c.n_total);
    const double cf = cos(th_f), sf = sin(th_f), cc = cos(th_c), sc = sin(th_c);
    const double cw = cos(th_w), sw = sin(th_w);
    col.dxx_e = c.d_perp + (c.dd * cf) * cf;
    col.dxy_e4 = 0.25 * ((c.dd * cf) * sf);
    col.dxx_w = c.d_perp + (c.dd * cw) * cw;
    col.dxy_w4 = 0.25 * ((c.dd * cw) * sw);
    col.dxy_c4 = 0.25 * ((c.dd * cc) * sc);
    col.dyy_c = c.d_perp + (c.dd * sc) * sc;
  }
  return col;
}

// Eq. (6) with one cross-lane exchange.  With the vertical second difference
// s = N + S - 2C of each column and r = C + s/6, the 9-point operator times
// dx^2 is
//   a_ax (W + E + N + S - 4C) + a_dg (NW + NE + SW + SE - 4C)
//     = (r_W + r_E - 2C) + (2/3) s,
// using a_ax + 2 a_dg = 1: only r crosses lanes (two shifts instead of four),
// and a constant field gives exactly zero (s = 0, r = C).
__device__ __forceinline__ double lap9_vertical(double up, double cen, double dn) {
  return fma(-2.0, cen, up + dn);  // 2C is exact: one rounding, as a subtraction
}
__device__ __forceinline__ double lap9_exchanged(double s, double cen) { return fma(kAlphaDiag, s, cen); }
__device__ __forceinline__ double lap9_combine(double rw, double re, double s, double cen, double coef) {
  return coef * fma(kAlphaAxial, s, fma(-2.0, cen, rw + re));
}

// Diffusion term at row `rho` of this lane's column, given the values `up`
// (row rho-1), `cen` (row rho) and `dn` (row rho+1), already mirrored in y
// (up = cen at rho = 0, dn = cen at rho = ny-1).  All lanes of the wave must
// call it together (cross-lane reads).  EDGE: some lane of this wave holds
// the first or last column of the grid, so x-mirrors must be applied.
// YEDGE = false promises 0 < rho < ny - 1 (no boundary face in y).
template <int STENCIL, bool EDGE, bool YEDGE = true>
__device__ __forceinline__ double diffusion(double up, double cen, double dn, const Column& col,
                                            int rho, const KConst& c, double coef) {
  if constexpr (STENCIL == RD_LAP5) {
    double w = from_west(cen), e = from_east(cen);
    if (EDGE && col.west) w = cen;
    if (EDGE && col.east) e = cen;
    return coef * (((w + e) + (up + dn)) - 4.0 * cen);
  } else if constexpr (STENCIL == RD_LAP9) {
    const double s = lap9_vertical(up, cen, dn);
    const double r = lap9_exchanged(s, cen);
    double rw = from_west(r), re = from_east(r);
    if (EDGE && col.west) rw = r;
    if (EDGE && col.east) re = r;
    return lap9_combine(rw, re, s, cen, coef);
  } else {
    // Conservative flux form: x-face fluxes shared with the west neighbour
    // through a lane shuffle, y-face fluxes recomputed by both rows with the
    // same operands; zero flux through boundary faces.
    const double wC = from_west(cen), eC = from_east(cen);
    const double wU = from_west(up), eU = from_east(up);
    const double wD = from_west(dn), eD = from_east(dn);
    double fxe = col.dxx_e * (eC - cen) + col.dxy_e4 * ((eD + dn) - (eU + up));
    if (EDGE && col.east) fxe = 0.0;
    double fxw = from_west(fxe);
    if (EDGE && col.west) fxw = 0.0;
    const bool mw = EDGE && col.west, me = EDGE && col.east;
    const double wCc = mw ? cen : wC, eCc = me ? cen : eC;
    const double wUc = mw ? up : wU, eUc = me ? up : eU;
    const double wDc = mw ? dn : wD, eDc = me ? dn : eD;
    double fys = col.dxy_c4 * ((eDc + eCc) - (wDc + wCc)) + col.dyy_c * (dn - cen);
    double fyn = col.dxy_c4 * ((eCc + eUc) - (wCc + wUc)) + col.dyy_c * (cen - up);
    if (YEDGE && !c.periodic && rho == c.ny - 1) fys = 0.0;
    if (YEDGE && !c.periodic && rho == 0) fyn = 0.0;
    return ((fxe - fxw) + (fys - fyn)) * coef;
  }
}

// The anisotropic flux form in a row sweep: the flux through the face north
// of row rho is the flux through the face south of row rho - 1, which the
// same stage computed one row earlier from the same operands in the same
// order.  CARRIED: take it from `fy` instead of recomputing it (the rows
// rho - 1 .. rho hold no y-boundary face).  `fy` receives this row's
// south-face flux for the next row.  Bit-identical to `diffusion`.
template <bool EDGE, bool YEDGE, bool CARRIED>
__device__ __forceinline__ double diffusion_flux_rows(double up, double cen, double dn, const Column& col,
                                                      int rho, const KConst& c, double coef, double& fy) {
  const double wC = from_west(cen), eC = from_east(cen);
  const double eU = from_east(up);
  const double wD = from_west(dn), eD = from_east(dn);
  double fxe = col.dxx_e * (eC - cen) + col.dxy_e4 * ((eD + dn) - (eU + up));
  if (EDGE && col.east) fxe = 0.0;
  double fxw = from_west(fxe);
  if (EDGE && col.west) fxw = 0.0;
  const bool mw = EDGE && col.west, me = EDGE && col.east;
  const double wCc = mw ? cen : wC, eCc = me ? cen : eC;
  const double wDc = mw ? dn : wD, eDc = me ? dn : eD;
  double fys = col.dxy_c4 * ((eDc + eCc) - (wDc + wCc)) + col.dyy_c * (dn - cen);
  double fyn;
  if constexpr (CARRIED) {
    fyn = fy;
  } else {
    const double wU = from_west(up);
    const double wUc = mw ? up : wU, eUc = me ? up : eU;
    fyn = col.dxy_c4 * ((eCc + eUc) - (wCc + wUc)) + col.dyy_c * (cen - up);
  }
  if (YEDGE && !c.periodic && rho == c.ny - 1) fys = 0.0;
  if (YEDGE && !c.periodic && rho == 0) fyn = 0.0;
  fy = fys;
  return ((fxe - fxw) + (fys - fyn)) * coef;
}

// The same operators with the three rows read from LDS.  Row arrays hold one
// value per lane at index lane + 1 (a pad column on each side); il is this
// lane's index, iw / ie the west / east neighbours after the x-mirror (equal
// to il where the neighbour is a ghost).  The arithmetic and its operand
// order are those of `diffusion`, so both give identical bits; the west
// x-face flux is recomputed here exactly as the west neighbour computes its
// east x-face flux.
template <int STENCIL, bool EDGE>
__device__ __forceinline__ double diffusion_rows(const double* up, const double* cen, const double* dn,
                                                 int il, int iw, int ie, const Column& col, int rho,
                                                 const KConst& c, double coef) {
  const double C = cen[il];
  if constexpr (STENCIL == RD_LAP5) {
    return coef * (((cen[iw] + cen[ie]) + (up[il] + dn[il])) - 4.0 * C);
  } else if constexpr (STENCIL == RD_LAP9) {
    // r of the neighbour columns, computed as those lanes compute their own
    const double rw = lap9_exchanged(lap9_vertical(up[iw], cen[iw], dn[iw]), cen[iw]);
    const double re = lap9_exchanged(lap9_vertical(up[ie], cen[ie], dn[ie]), cen[ie]);
    return lap9_combine(rw, re, lap9_vertical(up[il], C, dn[il]), C, coef);
  } else {
    const double u = up[il], d = dn[il];
    double fxe = col.dxx_e * (cen[il + 1] - C) + col.dxy_e4 * ((dn[il + 1] + d) - (up[il + 1] + u));
    if (EDGE && col.east) fxe = 0.0;
    double fxw = col.dxx_w * (C - cen[il - 1]) + col.dxy_w4 * ((d + dn[il - 1]) - (u + up[il - 1]));
    if (EDGE && col.west) fxw = 0.0;
    const double wCc = cen[iw], eCc = cen[ie], wUc = up[iw], eUc = up[ie], wDc = dn[iw], eDc = dn[ie];
    double fys = col.dxy_c4 * ((eDc + eCc) - (wDc + wCc)) + col.dyy_c * (d - C);
    double fyn = col.dxy_c4 * ((eCc + eUc) - (wCc + wUc)) + col.dyy_c * (C - u);
    if (!c.periodic && rho == c.ny - 1) fys = 0.0;
    if (!c.periodic && rho == 0) fyn = 0.0;
    return ((fxe - fxw) + (fys - fyn)) * coef;
  }
}

}  // namespace rd
