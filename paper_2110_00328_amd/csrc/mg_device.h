// mg_device.h -- per-cell arithmetic of the three scalar-field equations
// (Ruan et al., arXiv:2110.00328, Sec. 3.2.3-3.2.5) for gfx950, in two forms:
//
//  * direct form (the paper's nonlinear Gauss-Seidel): each cell of one
//    colour is replaced by the exact solution of its own discrete equation
//    with the six neighbours held fixed (eq:fR_eom_codeunit,
//    eq:sym_cubic_eqn) or by one Newton step (eq:relaxation_iteration, CQ);
//
//  * correction form (FP32 inner solves of the FP64-refined mode): the
//    unknown is the correction e about a frozen FP64 iterate x, the equation
//    is G(e) = F(x + e) - F(x) = rho, and every term of G is written so that
//    FP32 rounding is relative to e, not to x.  For f(R) the per-cell
//    equation becomes s^3 + (beta - 1 - gamma) s - beta = 0 in
//    s = sqrt(1 + e/x) and is polished in sigma = s - 1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgg {

enum { FR = 0, SYM = 1, CQ = 2 };

// Model constants in code units (Sec. 3.1.1), computed on the host in FP64.
struct Consts {
  int model;
  int cq_keep_exp;
  int fr_n;        // Hu-Sawicki n in {0, 1, 2}
  int pad_;
  double ct2;      // c~^2
  double om_a;     // Omega_m / a
  double K;        // R-bar(a) a^2 / 3 = Omega_m/a + 4 Omega_L a^2
  double wbar;     // |f_R(a)|
  double wpow;     // wbar^{1/(n+1)}
  double s_ratio;  // (a_*/a)^3
  double s_amp;    // a^2 / (2 xi^2)
  double ubar;     // sqrt(1 - (a_*/a)^3)
  double beta, alpha, phibar;
  double cq_src;   // 3 beta Omega_m a^-1 exp(beta phibar)
  double cq_pot;   // alpha lambda^2 a^2
  double cq_pb;    // phibar^-(1+alpha)
  double phi5;     // Phi5 prefactor: c~^2/2 (w), 3 xi^2 Om b*^2 c~^2 a*^-3 (u^2), beta (phi~)
  double bg;       // background value of the solved variable
  double bg_coef;  // |d| at the background per unit delta
  // FP32 copies used by the correction-form kernels
  float f_ct2, f_kw, f_s_ratio, f_s_amp, f_beta, f_alpha, f_phibar, f_cq_src, f_cq_pot;
  float f_i6ct2;     // 1 / (6 c~^2)
  float f_ict2;      // 1 / c~^2
  float f_isamp;     // 1 / s_amp
  float f_ct2_samp;  // c~^2 / s_amp
};

// ---------------------------------------------------------------------------
// math overloads
// ---------------------------------------------------------------------------
__device__ __forceinline__ double d_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float d_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double d_cbrt(double x) { return cbrt(x); }
__device__ __forceinline__ float d_cbrt(float x) { return cbrtf(x); }
__device__ __forceinline__ double d_sinh(double x) { return sinh(x); }
__device__ __forceinline__ float d_sinh(float x) { return sinhf(x); }
__device__ __forceinline__ double d_asinh(double x) { return asinh(x); }
__device__ __forceinline__ float d_asinh(float x) { return asinhf(x); }
__device__ __forceinline__ double d_cosh(double x) { return cosh(x); }
__device__ __forceinline__ float d_cosh(float x) { return coshf(x); }
__device__ __forceinline__ double d_acosh(double x) { return acosh(x); }
__device__ __forceinline__ float d_acosh(float x) { return acoshf(x); }
__device__ __forceinline__ double d_cos(double x) { return cos(x); }
__device__ __forceinline__ float d_cos(float x) { return cosf(x); }
__device__ __forceinline__ double d_acos(double x) { return acos(x); }
__device__ __forceinline__ float d_acos(float x) { return acosf(x); }
__device__ __forceinline__ double d_exp(double x) { return exp(x); }
__device__ __forceinline__ float d_exp(float x) { return expf(x); }
__device__ __forceinline__ double d_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float d_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double d_log1p(double x) { return log1p(x); }
__device__ __forceinline__ float d_log1p(float x) { return log1pf(x); }
__device__ __forceinline__ double d_pow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float d_pow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double d_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float d_rsqrt(float x) { return rsqrtf(x); }

// Hardware FP32 reciprocal, square root and reciprocal square root (single
// instructions, about 1 ulp) for the correction-form arithmetic, whose
// per-cell results are polished by Newton steps and whose FP32 inner
// problem only has to shrink the FP64-computed residual: the library's
// correctly rounded forms cost ten or more instructions each.
__device__ __forceinline__ float f_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float f_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float f_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float f_div(float a, float b) { return a * f_rcp(b); }

// Root of t^3 + p t + q = 0 on the branch the paper's closed forms select:
// the single real root, else the largest of three (for q < 0: the unique
// positive root).  Viete's trigonometric/hyperbolic forms -- Cardano's form
// cancels catastrophically when p^{3/2} >> |q| -- and one Newton step.
template <typename T>
__device__ __forceinline__ T cubic_root(T p, T q) {
  T t;
  if (p == T(0)) {
    t = d_cbrt(-q);
  } else if (p > T(0)) {
    T s = d_sqrt(p / T(3));
    T x = (T(1.5) * q / p) / s;
    t = T(-2) * s * d_sinh(d_asinh(x) / T(3));
  } else {
    T s = d_sqrt(-p / T(3));
    T x = (T(1.5) * q / p) / s;
    if (x >= T(1))
      t = T(2) * s * d_cosh(d_acosh(x) / T(3));
    else if (x <= T(-1))
      t = T(-2) * s * d_cosh(d_acosh(-x) / T(3));
    else
      t = T(2) * s * d_cos(d_acos(x) / T(3));
  }
  T f = (t * t + p) * t + q;
  T fp = T(3) * t * t + p;
  if (fp != T(0)) {
    T tn = t - f / fp;
    if (isfinite(tn)) t = tn;
  }
  return t;
}

// Approximation (relative error ~1e-5 away from double roots) of the same
// root from the hardware exp2/log2, for use as the start of Newton polishing:
//   sinh(asinh(x)/3) = (t - 1/t)/2,  cosh(acosh(x)/3) = (t + 1/t)/2,
//   t = (|x| + sqrt(x^2 +- 1))^{1/3}.
__device__ __forceinline__ float cubic_root_approx(float p, float q) {
  if (p == 0.0f) {
    float a = fabsf(q);
    float c = a > 0.0f ? __expf(__logf(a) * (1.0f / 3.0f)) : 0.0f;
    return q > 0.0f ? -c : c;
  }
  float s = f_sqrt(fabsf(p) * (1.0f / 3.0f));
  float x = f_div(1.5f * q, p * s);
  float ax = fabsf(x);
  if (p > 0.0f) {
    float y;
    if (ax < 1e-3f) {
      y = ax * (1.0f / 3.0f);
    } else {
      float L = ax > 1e18f ? __logf(2.0f * ax) : __logf(ax + f_sqrt(ax * ax + 1.0f));
      float t = __expf(L * (1.0f / 3.0f));
      y = 0.5f * (t - f_rcp(t));
    }
    return -2.0f * s * copysignf(y, x);
  }
  if (ax >= 1.0f) {
    float L = ax > 1e18f ? __logf(2.0f * ax) : __logf(ax + f_sqrt(ax * ax - 1.0f));
    float t = __expf(L * (1.0f / 3.0f));
    float y = 0.5f * (t + f_rcp(t));
    return copysignf(2.0f * s * y, x);
  }
  return 2.0f * s * __cosf(acosf(x) * (1.0f / 3.0f));
}

// FP64 root of t^3 + p t + q = 0 with q < 0 (unique positive root): FP32
// start, two FP64 Newton steps (quadratic from ~1e-5: ~1e-20); falls back to
// the FP64 closed form when the start is not usable.
__device__ __forceinline__ double cubic_root_pos64(double p, double q) {
  float t0 = cubic_root_approx(float(p), float(q));
  if (!(t0 > 0.0f) || !isfinite(t0)) return cubic_root<double>(p, q);
  double t = double(t0);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    double f = (t * t + p) * t + q;
    double fp = 3.0 * t * t + p;
    t -= f / fp;
  }
  return t;
}

// Unique positive root of u^2 + p u + q = 0 with q < 0 (eq:fR_quadratic_solns),
// in the rationalised form when p > 0 so that nothing cancels.
template <typename T>
__device__ __forceinline__ T quad_root_pos(T p, T q) {
  T sq = d_sqrt(p * p - T(4) * q);
  return p > T(0) ? T(-2) * q / (p + sq) : T(0.5) * (sq - p);
}

// Unique positive root of u^4 + p u + q = 0 with q < 0 (eq:fR_quartic_solns).
// The closed form loses all digits when |p| << |q|^{3/4}; instead Newton runs
// from an upper bound: f is convex for u > 0, so the iterates fall
// monotonically to the root.  Bounds: (-2q)^{1/4} always; -q/p when p > 0
// (then f(-q/p) = (q/p)^4 > 0); max((-2q)^{1/4}, (-2p)^{1/3}) when p < 0.
template <typename T>
__device__ __forceinline__ T quart_root_pos(T p, T q) {
  T u = d_sqrt(d_sqrt(T(-2) * q));
  if (p > T(0)) {
    T b = -q / p;
    if (b < u) u = b;
  } else if (p < T(0)) {
    T b = d_cbrt(T(-2) * p);
    if (b > u) u = b;
  }
  for (int it = 0; it < 64; ++it) {
    T u3 = u * u * u;
    T f = u3 * u + p * u + q;
    T fp = T(4) * u3 + p;
    if (!(fp > T(0))) break;
    T un = u - f / fp;
    if (!(un < u)) break;  // the monotone sequence has stopped
    u = un;
  }
  return u;
}

// w^{-1/(n+1)} of the f(R) nonlinearity
template <typename T>
__device__ __forceinline__ T fr_inv_root(int n, T w) {
  if (n == 1) return d_rsqrt(w);
  if (n == 0) return T(1) / w;
  return T(1) / d_cbrt(w);
}

// ---------------------------------------------------------------------------
// direct form: v <- exact per-cell solution of L^h(v)_c = S_c
// ---------------------------------------------------------------------------
// h2 = h^2 of the level (fine cell units), sum = sum of the six neighbours.
template <int M, typename T>
__device__ __forceinline__ T direct_update(const Consts& C, T h2, T vc, T sum, T dc, T sc) {
  if constexpr (M == FR) {
    // u^{n+2} + p u + q = 0, w = u^{n+1} (eq:fR_eom_codeunit; S shifts p)
    T g = h2 / (T(6) * T(C.ct2));
    T p = g * (T(C.om_a) * dc + T(C.K) - sc) - sum / T(6);
    T q = -g * T(C.K) * T(C.wpow);
    if (C.fr_n == 1) {
      T u;
      if constexpr (sizeof(T) == 8) u = cubic_root_pos64(p, q);
      else u = cubic_root<T>(p, q);
      return u * u;
    }
    if (C.fr_n == 0) return quad_root_pos<T>(p, q);
    T u = quart_root_pos<T>(p, q);
    return u * u * u;
  } else if constexpr (M == SYM) {
    // u^3 + p u + q = 0 (eq:sym_cubic_eqn; S shifts q)
    T kap = T(C.ct2) / (T(C.s_amp) * h2);
    T p = (T(1) + dc) * T(C.s_ratio) - T(1) + T(6) * kap;
    T q = -kap * sum + sc / T(C.s_amp);
    if constexpr (sizeof(T) == 8) {
      if (q < T(0)) return cubic_root_pos64(p, q);
    }
    return cubic_root<T>(p, q);
  } else {
    // Newton-Gauss-Seidel on eq:csf_eom_code
    T ct2 = T(C.ct2);
    T al = T(C.alpha);
    T x = C.cq_keep_exp ? T(C.beta) * vc / ct2 : T(0);
    T yb = vc / (ct2 * T(C.phibar));
    T lp = d_log1p(yb);
    T F = (sum - T(6) * vc) / h2 - T(C.cq_src) * (d_expm1(x) * (T(1) + dc) + dc) +
          T(C.cq_pot) * T(C.cq_pb) * d_expm1(-(T(1) + al) * lp) - sc;
    T ex = C.cq_keep_exp ? d_exp(x) : T(0);
    T dF = T(-6) / h2 - T(C.cq_src) * T(C.beta) / ct2 * ex * (T(1) + dc) -
           T(C.cq_pot) * (T(1) + al) / ct2 * T(C.cq_pb) / T(C.phibar) *
               d_exp(-(T(2) + al) * lp);
    return vc - F / dF;
  }
}

// direct form residual d = L^h(v)_c - S_c
template <int M, typename T>
__device__ __forceinline__ T direct_resid(const Consts& C, T h2, T vc, T sum, T dc, T sc) {
  T lap = (sum - T(6) * vc) / h2;
  if constexpr (M == FR) {
    return -T(C.ct2) * lap + T(C.om_a) * dc + T(C.K) -
           T(C.K) * T(C.wpow) * fr_inv_root<T>(C.fr_n, vc) - sc;
  } else if constexpr (M == SYM) {
    return T(C.ct2) * lap - T(C.s_amp) * (((T(1) + dc) * T(C.s_ratio) - T(1)) * vc + vc * vc * vc) - sc;
  } else {
    T ct2 = T(C.ct2);
    T x = C.cq_keep_exp ? T(C.beta) * vc / ct2 : T(0);
    T lp = d_log1p(vc / (ct2 * T(C.phibar)));
    return lap - T(C.cq_src) * (d_expm1(x) * (T(1) + dc) + dc) +
           T(C.cq_pot) * T(C.cq_pb) * d_expm1(-(T(1) + T(C.alpha)) * lp) - sc;
  }
}

// ---------------------------------------------------------------------------
// correction form (FP32): G(e)_c = F(x+e)_c - F(x)_c, solve G_c = rho_c
// ---------------------------------------------------------------------------
// expm1 and log1p for the tiny arguments of the correction form: the cubic
// Taylor polynomial below |z| < 1e-3 (relative error < 5e-11), the library
// function above.
__device__ __forceinline__ float expm1_small(float z) {
  return fabsf(z) < 1e-3f ? z * (1.0f + z * (0.5f + z * (1.0f / 6.0f))) : expm1f(z);
}
__device__ __forceinline__ float log1p_small(float z) {
  return fabsf(z) < 1e-3f ? z * (1.0f - z * (0.5f - z * (1.0f / 3.0f))) : log1pf(z);
}

// Coupled quintessence (eq:csf_eom_code) per cell, correction form: the
// change N(x+e) - N(x) of the non-Laplacian part, accurate relative to e, and
// its derivative dN/dv at x+e.  With Y = phibar + x/c^2, u = e/(c^2 Y),
// E1 = expm1(beta e/c^2), E2 = expm1(-(1+alpha) log1p(u)):
//   N(x+e) - N(x) = -src exp(beta x/c^2)(1+delta) E1 + pot Y^{-(1+alpha)} E2
//   dN/dv(x+e)    = -src (beta/c^2) exp(beta x/c^2)(1+E1)(1+delta)
//                   - pot ((1+alpha)/c^2) Y^{-(2+alpha)} (1+E2)/(1+u)
// The prefactors use the hardware exp/log (relative error ~1e-6, a scale
// factor only); the differences use expm1_small / log1p_small.
__device__ __forceinline__ void cq_corr_terms(const Consts& C, float x, float e, float dc,
                                              float* dn, float* dnp) {
  const float ict2 = C.f_ict2;
  const float a1 = 1.0f + C.f_alpha;
  const float Y = C.f_phibar + x * ict2;
  const float iY = f_rcp(Y);
  const float PX = __expf(-a1 * __logf(Y));  // Y^{-(1+alpha)}
  const float u = e * ict2 * iY;
  const float E2 = expm1_small(-a1 * log1p_small(u));
  float src = 0.0f, dsrc = 0.0f;
  if (C.cq_keep_exp) {
    const float ex = __expf(C.f_beta * x * ict2) * (1.0f + dc);
    const float E1 = expm1_small(C.f_beta * e * ict2);
    src = ex * E1;
    dsrc = C.f_beta * ict2 * ex * (1.0f + E1);
  }
  *dn = -C.f_cq_src * src + C.f_cq_pot * PX * E2;
  *dnp = -C.f_cq_src * dsrc - C.f_cq_pot * a1 * ict2 * (PX * iY) * (1.0f + E2) * f_rcp(1.0f + u);
}

// Nonlinear part N(x+e) - N(x) of each model, accurate relative to e.
template <int M>
__device__ __forceinline__ float corr_nl(const Consts& C, float e, float x, float dc) {
  if constexpr (M == FR) {
    // K wbar^m [x^{-m} - (x+e)^{-m}] = A [1 - (1+t)^{-m}], m = 1/(n+1),
    // t = e/x, A = K wbar^m x^{-m}; written without cancellation:
    //   n = 0: A t/(1+t);  n = 1: A t/(s(1+s)), s = sqrt(1+t);
    //   n = 2: A t/(c(c^2+c+1)), c = cbrt(1+t)
    float ix = f_rcp(x);
    float t = e * ix;
    if (C.fr_n == 1) {
      float s = f_sqrt(1.0f + t);
      return C.f_kw * f_rsq(x) * t * f_rcp(s * (1.0f + s));
    }
    if (C.fr_n == 0) return C.f_kw * ix * t * f_rcp(1.0f + t);
    float c = cbrtf(1.0f + t);
    return C.f_kw * f_rcp(cbrtf(x)) * t * f_rcp(c * ((c + 1.0f) * c + 1.0f));
  } else if constexpr (M == SYM) {
    // -s_amp [ (rho a*^3/a^3 - 1 + 3x^2) e + 3x e^2 + e^3 ]
    float m = (1.0f + dc) * C.f_s_ratio - 1.0f + 3.0f * x * x;
    return -C.f_s_amp * (m + (3.0f * x + e) * e) * e;
  } else {
    float dn, dnp;
    cq_corr_terms(C, x, e, dc, &dn, &dnp);
    return dn;
  }
}

// Laplacian coefficient kappa of each model: F = -kap Lap (f(R)), +kap Lap
// (symmetron, CQ); the sign is folded into corr_G.
template <int M>
__device__ __forceinline__ float corr_G(const Consts& C, float h2, float ec, float sum, float x,
                                        float dc) {
  float lap = (sum - 6.0f * ec) * (1.0f / h2);  // h2 = 4^l: exact
  if constexpr (M == FR) return -C.f_ct2 * lap + corr_nl<M>(C, ec, x, dc);
  else if constexpr (M == SYM) return C.f_ct2 * lap + corr_nl<M>(C, ec, x, dc);
  else return lap + corr_nl<M>(C, ec, x, dc);
}

// Exact per-cell solve of G_c(e) = rho with the neighbours fixed.
template <int M>
__device__ __forceinline__ float corr_update(const Consts& C, float h2, float ec_old, float sum,
                                             float x, float dc, float rho) {
  if constexpr (M == FR) {
    // D x t + A [1 - (1+t)^{-m}] = R,  D = 6c^2/h^2, R = rho + c^2 sum / h^2,
    // m = 1/(n+1).  With s = (1+t)^m:  s^{n+2} + (beta - 1 - gamma) s - beta = 0,
    //   beta = A / (D x), gamma = R / (D x);  sigma = s - 1 solves
    //   (1+sigma)^{n+2} - 1 + (beta - 1 - gamma) sigma - gamma = 0,
    //   whose linear coefficient is c1 = n + 1 + beta - gamma.
    const int n = C.fr_n;
    float iD = h2 * C.f_i6ct2;  // h^2 / (6 c^2), a level constant
    float ix = f_rcp(x);
    float xm = n == 1 ? ix * f_rsq(x) : (n == 0 ? ix * ix : ix * cbrtf(ix));  // x^{-(m+1)}
    float beta = C.f_kw * iD * xm;
    float gamma = (rho * iD + sum * (1.0f / 6.0f)) * ix;
    float c1 = float(n + 1) + beta - gamma;
    float sg;
    if (fabsf(gamma) < 1e-2f * c1) {
      sg = f_div(gamma, c1);  // small correction: linear guess, Newton below
    } else if (n == 1) {
      sg = cubic_root_approx(beta - 1.0f - gamma, -beta) - 1.0f;
    } else if (n == 0) {
      sg = quad_root_pos<float>(beta - 1.0f - gamma, -beta) - 1.0f;
    } else {
      sg = quart_root_pos<float>(beta - 1.0f - gamma, -beta) - 1.0f;
    }
    if (n == 1) {
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        float f = ((sg + 3.0f) * sg + c1) * sg - gamma;
        float fp = (3.0f * sg + 6.0f) * sg + c1;
        sg -= f_div(f, fp);
      }
      return x * sg * (sg + 2.0f);
    }
    if (n == 0) {
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        float f = (sg + c1) * sg - gamma;
        float fp = 2.0f * sg + c1;
        sg -= f_div(f, fp);
      }
      return x * sg;
    }
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      float f = (((sg + 4.0f) * sg + 6.0f) * sg + c1) * sg - gamma;
      float fp = ((4.0f * sg + 12.0f) * sg + 12.0f) * sg + c1;
      sg -= f_div(f, fp);
    }
    return x * sg * ((sg + 3.0f) * sg + 3.0f);
  } else if constexpr (M == SYM) {
    // e^3 + 3x e^2 + P e + Q = 0, P = m + 6 kap, Q = rho/s_amp - kap sum,
    // m = (1+delta) a*^3/a^3 - 1 + 3x^2, kap = c^2/(s_amp h^2)
    float kap = C.f_ct2_samp * (1.0f / h2);
    // 6 kap is a level constant: added with explicit rounding so that no
    // kernel fuses it into the sum and another not
    float P = __fadd_rn((1.0f + dc) * C.f_s_ratio - 1.0f + 3.0f * x * x, __fmul_rn(6.0f, kap));
    float Q = rho * C.f_isamp - kap * sum;
    float e;
    if (P > 0.0f && fabsf(Q) < 1e-2f * P * fabsf(x)) {
      e = f_div(-Q, P);
    } else {
      // total field y = x + e solves y^3 + p y + q = 0 (paper's branch)
      float p = P - 3.0f * x * x;
      float q = (2.0f * x * x - P) * x + Q;
      e = (q < 0.0f ? cubic_root_approx(p, q) : cubic_root<float>(p, q)) - x;
    }
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      float g = ((e + 3.0f * x) * e + P) * e + Q;
      float gp = (3.0f * e + 6.0f * x) * e + P;
      if (gp != 0.0f) e -= f_div(g, gp);
    }
    return e;
  } else {
    // Newton-Gauss-Seidel (eq:relaxation_iteration) on the correction
    float dn, dnp;
    cq_corr_terms(C, x, ec_old, dc, &dn, &dnp);
    const float ih2 = 1.0f / h2;  // h2 = 4^l: exact
    float G = (sum - 6.0f * ec_old) * ih2 + dn - rho;
    float dG = -6.0f * ih2 + dnp;
    return ec_old - f_div(G, dG);
  }
}

// Four consecutive cells of corr_update.  f(R) n = 1, the hot case, takes
// all four through the same steps so that the common small-correction path
// has no per-cell branch: every cell gets the linear guess, the closed-form
// start replaces it only where the correction is large, then all four take
// the two Newton steps together.  Same arithmetic as corr_update.
template <int M>
__device__ __forceinline__ void corr_update4(const Consts& C, float h2, const float* eo,
                                             const float* sum, const float* x, const float* dc,
                                             const float* rho, float* out) {
  if constexpr (M == FR) {
    if (C.fr_n == 1) {
      const float iD = h2 * C.f_i6ct2;
      float gamma[4], c1[4], sg[4], beta[4];
      bool big = false;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float ix = f_rcp(x[q]);
        beta[q] = C.f_kw * iD * (ix * f_rsq(x[q]));
        gamma[q] = (rho[q] * iD + sum[q] * (1.0f / 6.0f)) * ix;
        c1[q] = 2.0f + beta[q] - gamma[q];
        sg[q] = f_div(gamma[q], c1[q]);
        big |= !(fabsf(gamma[q]) < 1e-2f * c1[q]);
      }
      if (big) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (!(fabsf(gamma[q]) < 1e-2f * c1[q]))
            sg[q] = cubic_root_approx(beta[q] - 1.0f - gamma[q], -beta[q]) - 1.0f;
      }
#pragma unroll
      for (int it = 0; it < 2; ++it)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float f = ((sg[q] + 3.0f) * sg[q] + c1[q]) * sg[q] - gamma[q];
          const float fp = (3.0f * sg[q] + 6.0f) * sg[q] + c1[q];
          sg[q] -= f_div(f, fp);
        }
#pragma unroll
      for (int q = 0; q < 4; ++q) out[q] = x[q] * sg[q] * (sg[q] + 2.0f);
      return;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = corr_update<M>(C, h2, eo[q], sum[q], x[q], dc[q], rho[q]);
}

// d G_c / d e_c (diagonal of the correction operator; used by the uniform-
// mode Newton step of the coarsest CQ level)
template <int M>
__device__ __forceinline__ float corr_diag(const Consts& C, float h2, float ec, float x, float dc) {
  if constexpr (M == CQ) {
    float dn, dnp;
    cq_corr_terms(C, x, ec, dc, &dn, &dnp);
    return -6.0f / h2 + dnp;
  } else {
    return 1.0f;
  }
}

// direct-form diagonal dF_c/dv_c (uniform-mode Newton step, CQ)
template <int M, typename T>
__device__ __forceinline__ T direct_diag(const Consts& C, T h2, T vc, T dc) {
  if constexpr (M == CQ) {
    T ct2 = T(C.ct2);
    T ex = C.cq_keep_exp ? d_exp(T(C.beta) * vc / ct2) : T(0);
    T Y = T(C.phibar) + vc / ct2;
    return T(-6) / h2 - T(C.cq_src) * T(C.beta) / ct2 * ex * (T(1) + dc) -
           T(C.cq_pot) * (T(1) + T(C.alpha)) / ct2 * d_pow(Y, -(T(2) + T(C.alpha)));
  } else {
    return T(1);
  }
}

// ---------------------------------------------------------------------------
// Linearised operator for the adjoint:  J = s A,
//   A v = kap (6 v - sum v)/h^2 + dg_c v   (symmetric positive definite)
// ---------------------------------------------------------------------------
// kap and s per model; dg_c and dF_c/ddelta_c from the converged field.
__host__ __device__ __forceinline__ double lin_kap(const Consts& C) {
  return C.model == CQ ? 1.0 : C.ct2;
}
__host__ __device__ __forceinline__ double lin_sign(const Consts& C) {
  return C.model == FR ? 1.0 : -1.0;
}

template <int M>
__device__ __forceinline__ double lin_dg(const Consts& C, double v, double dc) {
  if constexpr (M == FR) {
    // m K wbar^m w^{-m-1}, m = 1/(n+1)
    if (C.fr_n == 1) return 0.5 * C.K * C.wpow * pow(v, -1.5);
    if (C.fr_n == 0) return C.K * C.wpow / (v * v);
    return C.K * C.wpow / 3.0 * pow(v, -4.0 / 3.0);
  } else if constexpr (M == SYM) {
    return C.s_amp * (((1.0 + dc) * C.s_ratio - 1.0) + 3.0 * v * v);
  } else {
    double ex = C.cq_keep_exp ? exp(C.beta * v / C.ct2) : 0.0;
    return C.cq_src * C.beta / C.ct2 * ex * (1.0 + dc) +
           C.cq_pot * (1.0 + C.alpha) / C.ct2 * pow(C.phibar + v / C.ct2, -(2.0 + C.alpha));
  }
}

template <int M>
__device__ __forceinline__ double lin_dfd(const Consts& C, double v) {
  if constexpr (M == FR) return C.om_a;
  else if constexpr (M == SYM) return -C.s_amp * C.s_ratio * v;
  else return -C.cq_src * (C.cq_keep_exp ? exp(C.beta * v / C.ct2) : 1.0);
}

}  // namespace mgg
