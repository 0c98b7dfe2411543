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

// e * 2^k as a pair for an integer e (|e| < 2^11 keeps e * LN2_A exact;
// beyond, the product pair is exact anyway)
LMH_INLINE ddd ln2_times(double e) { return dd2_add2(dd2_mul(e, LN2_A_D), e * LN2_B_D); }

// pow partials for finite x != 0 (x < 0 with integer y for gx), finite y:
// with g = gm 2^ge, y = ym 2^ye and log|x| = lm 2^le (gm, ym, lm in [0.5,
// 1)), the power-of-two exponents join the exponential's argument,
//   gx = gm ym e^((y - 1) log|x| + (ye + ge) ln2),
//   gy = gm lm e^(y log|x| + (le + ge) ln2),
// so every product stays near 1 and each partial is rounded once by the
// final scaling, however large or small g, y and the power are (the clamp of
// the exponential's argument at +-1000 is then exactly overflow / underflow).
LMH_INLINE void pow_bwd(double x, double y, double g, double& gx, double& gy) {
  double ax = fabs_(x);
  ddd lg = log_dd(ax);
  double gm = frexp_mant_(g), ym = frexp_mant_(y);
  double ge = (double)frexp_exp_(g), ye = (double)frexp_exp_(y);
  int ile = frexp_exp_(lg.hi);
  ddd lm = mk(ldexp_(lg.hi, -ile), ldexp_(lg.lo, -ile));
  ddd w = dd2_mul(lg, y);                                  // y log|x|
  double k1, k2;
  ddd e1 = exp_dd(dd2_add2(dd2_add2(w, dd2_neg(lg)), ln2_times(ye + ge)), k1);
  ddd e2 = exp_dd(dd2_add2(w, ln2_times((double)ile + ge)), k2);
  double dx = dd_ldexp(dd2_mul(dd2_mul(e1, ym), gm), (int)k1);
  double dy = dd_ldexp(dd2_mul(dd2_mul(e2, lm), gm), (int)k2);
  bool yint = rint_(y) == y;
  bool ym1odd = yint && fabs_(y) < 0x1p53 && !is_odd_int(y);   // y - 1 odd
  dx = (x < 0.0 && ym1odd) ? -dx : dx;                     // x^(y-1) = -|x|^(y-1)
  dy = x < 0.0 ? __builtin_nan("") : dy;
  // x = +-0, infinite or NaN, and x < 0 with y not an integer: the forward
  // pow, which carries every Annex F case
  bool plain = ax != 0.0 && isfinite_(ax) && isfinite_(y) && (x > 0.0 || yint);
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

LMH_INLINE fff ln2_timesf(float e) { return dd2_add2(dd2_mul(e, LN2_HI_F), e * LN2_LO_F); }

// as the binary64 form; the exponential's argument is clamped at +-110, where
// the result (a pair below 1.42 times e^-110) is below half the smallest
// subnormal, or (1/8 e^110) overflows
LMH_INLINE void pow_bwd(float x, float y, float g, float& gx, float& gy) {
  float ax = fabs_(x);
  fff lg = logf_ff(ax);
  float gm = frexp_mant_(g), ym = frexp_mant_(y);
  float ge = (float)frexp_exp_(g), ye = (float)frexp_exp_(y);
  int ile = frexp_exp_(lg.hi);
  fff lm = mk(ldexp_(lg.hi, -ile), ldexp_(lg.lo, -ile));
  fff w = dd2_mul(lg, y);
  float k1, k2;
  fff e1 = expf_ff(dd2_add2(dd2_add2(w, dd2_neg(lg)), ln2_timesf(ye + ge)), k1, 110.0f);
  fff e2 = expf_ff(dd2_add2(w, ln2_timesf((float)ile + ge)), k2, 110.0f);
  float dx = ff_ldexp(dd2_mul(dd2_mul(e1, ym), gm), (int)k1);
  float dy = ff_ldexp(dd2_mul(dd2_mul(e2, lm), gm), (int)k2);
  bool yint = rint_(y) == y;
  bool ym1odd = yint && fabs_(y) < 0x1p24f && !is_odd_intf(y);
  dx = (x < 0.0f && ym1odd) ? -dx : dx;
  dy = x < 0.0f ? __builtin_nanf("") : dy;
  bool plain = ax != 0.0f && isfinite_(ax) && isfinite_(y) && (x > 0.0f || yint);
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
