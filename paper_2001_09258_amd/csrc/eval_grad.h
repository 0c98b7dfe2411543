// Backward (vector-Jacobian) evaluators: g * f'(x), formed from the forward
// evaluators' double-double / float-float pieces so that each gradient is
// rounded once where the derivative allows it:
//
//   sin' = cos, cos' = -sin, exp' = exp (one extra rounding: the product),
//   tan' = 1 + tan^2 (from the unrounded tan pair), log' = 1/x (IEEE division),
//   tanh' = sech^2 = 1/cosh^2 (computed as g / C^2 * 2^-2k with
//           cosh = C 2^k, so large |x| underflows gracefully instead of
//           overflowing cosh^2; no 1 - tanh^2 cancellation),
//   pow:  d/dx = g y x^(y-1) = g y e^((y-1) log x),  d/dy = g x^y log x,
//   atan2: d/dy = g x / (x^2 + y^2), d/dx = -g y / (x^2 + y^2), with x, y
//          scaled by a common power of two first so the squares cannot
//          overflow or underflow.
#pragma once
#include "eval_f64.h"
#include "eval_f32.h"
#pragma STDC FP_CONTRACT OFF

namespace lmh {

// ---- binary64 --------------------------------------------------------------
LMH_INLINE double sin_bwd(double x, double g) { return g * cos_u10(x); }
LMH_INLINE double cos_bwd(double x, double g) { return -(g * sin_u10(x)); }
LMH_INLINE double exp_bwd(double x, double g) { return g * exp_u10(x); }
LMH_INLINE double log_bwd(double x, double g) { return g / x; }
LMH_INLINE double tan_bwd(double x, double g) {
  ddd t = tan_dd(x);
  ddd d = dd2_add(1.0, dd2_squ(t));                        // 1 + tan^2 >= 1
  ddd r = dd2_mul(d, g);
  return r.hi + r.lo;
}

// cosh(|x|) = C * 2^k with C a pair in about [0.5, 2]
LMH_INLINE ddd cosh_scaled(double ax, double& k) {
  ddd e = exp_half(ax > 711.0 ? 711.0 : ax, k);            // e^ax / 2 = e 2^k
  ddd rc = dd2_rec(e);                                     // 2 e^-ax 2^k
  ddd g = mk(ldexp_(rc.hi, -2 * (int)k - 2), ldexp_(rc.lo, -2 * (int)k - 2));
  return dd2_add(e, g);                                    // (cosh) 2^-k
}

LMH_INLINE double tanh_bwd(double x, double g) {
  double k;
  ddd c = cosh_scaled(fabs_(x), k);
  ddd q = dd2_div(mk(g, 0.0), dd2_squ(c));
  double r = dd_ldexp(q, -2 * (int)k);
  return isnan_(x) ? x : r;
}

LMH_INLINE void pow_bwd(double x, double y, double g, double& gx, double& gy) {
  double ax = fabs_(x);
  ddd lg = log_dd(ax);
  ddd w = dd2_mul(lg, y);                                  // y log x
  double k1, k2;
  ddd e1 = exp_dd(dd2_add2(w, dd2_neg(lg)), k1);           // x^(y-1)
  ddd e2 = exp_dd(w, k2);                                  // x^y
  double dx = dd_ldexp(dd2_mul(dd2_mul(e1, y), g), (int)k1);
  double dy = dd_ldexp(dd2_mul(dd2_mul(e2, lg), g), (int)k2);
  bool yint = rint_(y) == y;
  bool ym1odd = yint && fabs_(y) < 0x1p53 && !is_odd_int(y);   // y-1 odd
  dx = (x < 0.0 && ym1odd) ? -dx : dx;
  // outside x > 0 (and for overflowing magnitudes) use the forward pow,
  // which carries every Annex F case
  bool plain = x > 0.0 && isfinite_(x) && isfinite_(y) && fabs_(w.hi) < 700.0;
  if (!plain) {
    dx = g * (y * pow_u10(x, y - 1.0));
    dy = x > 0.0 ? g * (pow_u10(x, y) * (lg.hi + lg.lo)) : __builtin_nan("");
    dy = (x == 0.0 && y >= 0.0) ? 0.0 : dy;
    dx = (y == 0.0) ? 0.0 : dx;
  }
  gx = dx;
  gy = dy;
}

LMH_INLINE void atan2_bwd(double y, double x, double g, double& gy, double& gx) {
  double m = fabs_(x) > fabs_(y) ? fabs_(x) : fabs_(y);
  int k = frexp_exp_(m);
  double xs = ldexp_(x, -k), ys = ldexp_(y, -k);
  ddd d = dd2_add2(dd2_mul(xs, xs), dd2_mul(ys, ys));      // in [1/4, 2)
  gy = dd_ldexp(dd2_div(dd2_mul(g, xs), d), -k);
  gx = dd_ldexp(dd2_div(dd2_mul(-g, ys), d), -k);
}

// ---- binary32 --------------------------------------------------------------
LMH_INLINE float sin_bwd(float x, float g) { return g * cosf_u10(x); }
LMH_INLINE float cos_bwd(float x, float g) { return -(g * sinf_u10(x)); }
LMH_INLINE float exp_bwd(float x, float g) { return g * expf_u10(x); }
LMH_INLINE float log_bwd(float x, float g) { return g / x; }
LMH_INLINE float tan_bwd(float x, float g) {
  fff t = tanf_ff(x);
  fff d = dd2_add(1.0f, dd2_squ(t));
  fff r = dd2_mul(d, g);
  return r.hi + r.lo;
}

LMH_INLINE fff coshf_scaled(float ax, float& k) {
  fff e = expf_half(ax > 90.0f ? 90.0f : ax, k);
  fff rc = dd2_rec(e);
  fff g = mk(ldexp_(rc.hi, -2 * (int)k - 2), ldexp_(rc.lo, -2 * (int)k - 2));
  return dd2_add(e, g);
}

LMH_INLINE float tanh_bwd(float x, float g) {
  float k;
  fff c = coshf_scaled(fabs_(x), k);
  fff q = dd2_div(mk(g, 0.0f), dd2_squ(c));
  float r = ff_ldexp(q, -2 * (int)k);
  return isnan_(x) ? x : r;
}

LMH_INLINE void pow_bwd(float x, float y, float g, float& gx, float& gy) {
  float ax = fabs_(x);
  fff lg = logf_ff(ax);
  fff w = dd2_mul(lg, y);
  float k1, k2;
  fff e1 = expf_ff(dd2_add2(w, dd2_neg(lg)), k1);
  fff e2 = expf_ff(w, k2);
  float dx = ff_ldexp(dd2_mul(dd2_mul(e1, y), g), (int)k1);
  float dy = ff_ldexp(dd2_mul(dd2_mul(e2, lg), g), (int)k2);
  bool yint = rint_(y) == y;
  bool ym1odd = yint && fabs_(y) < 0x1p24f && !is_odd_intf(y);
  dx = (x < 0.0f && ym1odd) ? -dx : dx;
  bool plain = x > 0.0f && isfinite_(x) && isfinite_(y) && fabs_(w.hi) < 85.0f;
  if (!plain) {
    dx = g * (y * powf_u10(x, y - 1.0f));
    dy = x > 0.0f ? g * (powf_u10(x, y) * (lg.hi + lg.lo)) : __builtin_nanf("");
    dy = (x == 0.0f && y >= 0.0f) ? 0.0f : dy;
    dx = (y == 0.0f) ? 0.0f : dx;
  }
  gx = dx;
  gy = dy;
}

LMH_INLINE void atan2_bwd(float y, float x, float g, float& gy, float& gx) {
  float m = fabs_(x) > fabs_(y) ? fabs_(x) : fabs_(y);
  int k = frexp_exp_(m);
  float xs = ldexp_(x, -k), ys = ldexp_(y, -k);
  fff d = dd2_add2(dd2_mul(xs, xs), dd2_mul(ys, ys));
  gy = ff_ldexp(dd2_div(dd2_mul(g, xs), d), -k);
  gx = ff_ldexp(dd2_div(dd2_mul(-g, ys), d), -k);
}

}  // namespace lmh

#pragma STDC FP_CONTRACT DEFAULT
