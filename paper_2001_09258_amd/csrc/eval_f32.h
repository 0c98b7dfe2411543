// Binary32 evaluators.  The paper covers binary64 only; these follow the same
// reduction / polynomial / reconstruction structure in binary32, with
// float-float pairs only where the 1-ULP bound needs them (the reduced
// argument, the lowest polynomial terms, the reconstructions).  Binary64
// arithmetic appears only on lanes whose result is subnormal, where
// float-float cannot decide the one rounding (exp, exp2, exp10, pow: see
// f32_sub_units; hypot: see hypotf_u10_main), and in four C99 additions that
// evaluate in binary64 working precision and round once: erf, erfc, lgamma
// and tgamma.
#pragma once
#include "dd.h"
#include "generated/consts.inc"
#include "generated/poly_coeffs.inc"
#include "generated/ph_table_f32.inc"
#include "eval_f64.h"                          // binary64 pieces used in working precision
#pragma STDC FP_CONTRACT OFF

namespace lmh {

typedef dd2<float> fff;

// v * 2^q correctly rounded into binary32, including subnormal results
LMH_INLINE float ff_ldexp(fff v, int q) {
  float r = ldexp_(v.hi + v.lo, q);
  if (q < -122) {
    v = dd2_norm(v);                                // |lo| <= ulp(hi)/2
    float h = ldexp_(v.hi, q + 149);
    float l = ldexp_(v.lo, q + 149);
    float n = rint_(h);
    float d = (h - n) + l;
    n = d > 0.5f ? n + 1.0f : (d < -0.5f ? n - 1.0f : n);
    float s = ldexp_(n, -149);
    r = fabs_(h) < 0x1p23f ? s : r;
  }
  return r;
}

// Binary32 results in the subnormal range (below 2^-126) keep up to 23 bits,
// and deciding the last one needs the value to well below 2^-23 of a
// subnormal ulp.  The working float-float paths reach ~2^-30 relative (one
// subnormal result in a few thousand came out a unit off), and float-float
// cannot go much below 2^-46, which would still leave an expected miss over
// the 2^21 binary32 inputs whose exp is subnormal.  So the lanes whose
// result falls in that range evaluate the binary64 pieces (~2^-60) and round
// once here: v 2^q in units of 2^-149, rounded to an integer with the low
// word deciding; d is the distance from rint(hi) in those units.
LMH_INLINE double f32_sub_units(ddd v, int q, double& d) {
  v = dd2_norm(v);
  double h = ldexp_(v.hi, q + 149);
  double l = ldexp_(v.lo, q + 149);
  double n = rint_(h);
  d = (h - n) + l;
  return d > 0.5 ? n + 1.0 : (d < -0.5 ? n - 1.0 : n);
}

LMH_INLINE float f32_from_units(double n) { return ldexp_((float)n, -149); }

LMH_INLINE bool is_odd_intf(float q) { return q - 2.0f * rint_(q * 0.5f) != 0.0f; }

// ---------------------------------------------------------------------------
// exp family
// ---------------------------------------------------------------------------
LMH_INLINE fff expf_core(float rh, float rl) {
  float p = poly_estrin(rh, EXP_P_F32);
  float w = fma_(rh * rh, p, fma_(rl, rh, rl));
  fff s = dd2_add(1.0f, rh);
  return mk(s.hi, s.lo + w);
}

// (F_main / F_rare / F as in eval_f64.h: the rare path decides results in
// the subnormal range)
LMH_INLINE float expf_u10_main(float x, bool& rare) {
  // beyond +-104 the result overflows / rounds to zero; the clamp keeps
  // k * LN2_HI exact (|k| <= 150)
  float xc = x > 104.0f ? 104.0f : (x < -104.0f ? -104.0f : x);
  float k = rint_(xc * LOG2E_F);
  float s = fma_(k, -LN2_HI_F, xc);
  float t = k * -LN2_LO_F;
  float rh = s + t;
  float rl = (s - rh) + t;
  fff e = expf_core(rh, rl);
  // results below 2^-125 (the pair is in [0.7, 1.42]); a clamped argument
  // (x < -104, e^x < 2^-150) rounds to zero on this path
  rare = k <= -126.0f && x >= -104.0f;
  float r = ldexp_(e.hi + e.lo, (int)k);
  return isnan_(x) ? x : r;
}

LMH_INLINE float expf_u10_rare(float x) {          // -104 <= x < -87
  double sh, sl, d;
  double kd = exp_reduce((double)x, sh, sl);
  return f32_from_units(f32_sub_units(exp_core(sh, sl), (int)kd, d));
}

LMH_INLINE float expf_u10(float x) {
  bool rare;
  float r = expf_u10_main(x, rare);
  if (rare_lane(rare)) {
    float rs = expf_u10_rare(rare ? x : -95.0f);
    r = rare ? rs : r;
  }
  return r;
}

LMH_INLINE float exp2f_u10_main(float x, bool& rare) {
  float xc = x > 150.0f ? 150.0f : (x < -150.0f ? -150.0f : x);
  float k = rint_(xc);
  float f = xc - k;
  fff t = dd2_mul(f, LN2_F_H);
  t.lo = fma_(f, LN2_F_L, t.lo);
  t = dd2_norm(t);
  fff e = expf_core(t.hi, t.lo);
  // x <= -150 gives 2^-150 or less: zero (the tie at -150 to even)
  rare = k <= -126.0f && x > -150.0f;
  float r = ldexp_(e.hi + e.lo, (int)k);
  return isnan_(x) ? x : r;
}

LMH_INLINE float exp2f_u10_rare(float x) {         // -150 < x < -125.5
  float k = rint_(x);
  double fd = (double)(x - k), d;                   // exact
  ddd td = dd2_norm(dd2_add2(dd2_mul(fd, LN2_D_H), dd2_mul(fd, LN2_D_L)));
  return f32_from_units(f32_sub_units(exp_core(td.hi, td.lo), (int)k, d));
}

LMH_INLINE float exp2f_u10(float x) {
  bool rare;
  float r = exp2f_u10_main(x, rare);
  if (rare_lane(rare)) {
    float rs = exp2f_u10_rare(rare ? x : -140.0f);
    r = rare ? rs : r;
  }
  return r;
}

LMH_INLINE fff expf_ff(fff w, float& k, float lim = 104.0f) {
  float wh = w.hi > lim ? lim : (w.hi < -lim ? -lim : w.hi);
  float wl = wh == w.hi ? w.lo : 0.0f;              // the tail goes with a clamp
  k = rint_(wh * LOG2E_F);
  float s = fma_(k, -LN2_HI_F, wh);
  fff r = dd2_add2(s, wl + k * -LN2_LO_F);
  return dd2_norm(expf_core(r.hi, r.lo));
}

// ---------------------------------------------------------------------------
// log family: a = m 2^e, m in [0.75, 1.5), t = (m-1)/(m+1) as a float pair
// ---------------------------------------------------------------------------
LMH_INLINE fff logf_t(float a, float& e) {
  float m = frexp_mant_(a);
  int ie = frexp_exp_(a);
  bool low = m < 0.75f;
  m = low ? m + m : m;
  e = (float)(low ? ie - 1 : ie);
  fff den = dd2_add(1.0f, m);                        // fast two-sum: m < 2
  return dd2_div(mk(m - 1.0f, 0.0f), den);
}

LMH_INLINE float logf_u10(float x) {
  float e;
  fff t = logf_t(x, e);
  float z = t.hi * t.hi;
  float q = poly_estrin(z, LOG_Q_F32);
  float t3q = (t.hi * z) * q;
  fff s = dd2_add2(e * LN2_HI_F, t.hi + t.hi);
  float r = s.hi + (s.lo + (e * LN2_LO_F + ((t.lo + t.lo) + t3q)));
  r = x == 0.0f ? -__builtin_inff() : r;
  r = x < 0.0f ? __builtin_nanf("") : r;
  r = (isinf_(x) && x > 0.0f) || isnan_(x) ? x : r;
  return r;
}

LMH_INLINE float logf_u35(float x) {
  float m = frexp_mant_(x);
  int ie = frexp_exp_(x);
  bool low = m < 0.75f;
  m = low ? m + m : m;
  float e = (float)(low ? ie - 1 : ie);
  float t = (m - 1.0f) / (m + 1.0f);
  float z = t * t;
  float lm = fma_(t * z, poly_estrin(z, LOG_Q_F32), t + t);
  float r = fma_(e, LN2_HI_F, fma_(e, LN2_LO_F, lm));
  r = x == 0.0f ? -__builtin_inff() : r;
  r = x < 0.0f ? __builtin_nanf("") : r;
  r = (isinf_(x) && x > 0.0f) || isnan_(x) ? x : r;
  return r;
}

LMH_INLINE float log2f_u10(float x) {
  float e;
  fff t = logf_t(x, e);
  float z = t.hi * t.hi;
  float q = poly_estrin(z, LOG_Q_F32);
  float t3q = (t.hi * z) * q;
  fff lm = dd2_add(t.hi + t.hi, (t.lo + t.lo) + t3q);
  fff l2 = dd2_mul(lm, mk(INVLN2_F_H, INVLN2_F_L));
  fff s = dd2_add2(e, l2.hi);
  float r = s.hi + (s.lo + l2.lo);
  r = x == 0.0f ? -__builtin_inff() : r;
  r = x < 0.0f ? __builtin_nanf("") : r;
  r = (isinf_(x) && x > 0.0f) || isnan_(x) ? x : r;
  return r;
}

// ---------------------------------------------------------------------------
// trigonometric reductions in binary32
// ---------------------------------------------------------------------------
// Cody-Waite for |x| < 65536 in float-float (binary32 arithmetic only):
// r = x - q C with C = c0 + c1 + c2 + c3 (c0 the nearest float, c1 the rest
// to 8 significant bits, c2 and c3 nearest floats; together within 2^-78
// of C), |q| < 2^16.
// * x - q c0 is exact, so one FMA forms it: both are multiples of the last
//   place of c0 or of x (|x| >= 1/2 wherever q != 0), and the difference is
//   below 2 (C = pi) or 1 (C = pi/2) in magnitude, 24 bits.  cos's q = +-1
//   meets |x| < 1, where the difference is not exact: ODD_HEAD adds the
//   two-sum error there (q c0 = +-c0 is exact).
// * q c1 is exact (at most 16 + 8 bits) and r0 - q c1 is a two-sum; q c2,
//   below 2^-17, is an exact FMA pair whose head is a second two-sum.
// * The low words left are added rounded.  Where r is small, s is within
//   2^-17 of r, so every low word is below 2^-40 and the error about 2^-64
//   absolute, against a reduced argument of at least 2^-27.8 for
//   |x| < 65536 (the float nearest to 161 pi/2); elsewhere the low words are
//   below 2^-24 |r| and the error below 2^-47 |r|.
template <bool ODD_HEAD>
LMH_INLINE fff cwf_reduce(float x, float q, float c0, float c1, float c2, float c3) {
  float r0 = fma_(q, -c0, x);
  float e0 = 0.0f;
  if (ODD_HEAD) {
    float qc = q * -c0;                           // exact for q = +-1
    float v = r0 - x;
    e0 = fabs_(x) < 1.0f ? (x - (r0 - v)) + (qc - v) : 0.0f;
  }
  fff s = dd2_add2(r0, q * -c1);
  fff p2 = dd2_mul(q, -c2);
  fff t = dd2_add2(s.hi, p2.hi);
  float lo = ((s.lo + t.lo) + e0) + fma_(q, -c3, p2.lo);
  return dd2_add(t.hi, lo);
}

// Payne-Hanek in binary32, the binary64 core's steps in float-float:
// |x| = m 2^(ex-23), m < 2^24 an integer; row e of the table holds
// (2^(e-23) 2/pi) mod 4 in four 23-bit fixed-position limbs (limb i: the
// weights 2^(1-23i) .. 2^(-21-23i)), row ex for 2|x|/pi, row ex-1 for
// |x|/pi.  Returns f = rfrac(m W + h) as a pair, |f| <= 1/2 + 2^-19, and j
// congruent modulo 4 to the integer removed.  Exactness, with the binary64
// argument's numbers scaled: m w0 is a multiple of 2^-21 below 2^26 and
// m w1 one of 2^-44 below 8 (exact pairs), x0 and t - rint t are exact, e + p1
// is a multiple of 2^-44 below 2^-20 (exact), and the normalising fast
// two-sum is exact (where the low part is the larger, every difference it
// forms is a multiple of 2^-44 below 2^-20); m w2 < 2^-20 is an exact pair
// and m w3 < 2^-43 is rounded once (2^-67, the size of the table's
// truncation times m, 2^-66).
LMH_INLINE fff phf_core(float a, int row_shift, float h, float& j) {
  int ex = frexp_exp_(a) - 1;
  int row = ex - row_shift;
  row = row < 0 ? 0 : (row > 127 ? 127 : row);
  float m = ldexp_(frexp_mant_(a), 24);
  const float* W = PH_TABLE_F32 + 4 * row;
  fff p0 = dd2_mul(m, W[0]);
  float i0 = rint_(p0.hi), j0 = rint_(p0.lo);
  float x0 = ((p0.hi - i0) + (p0.lo - j0)) + h;
  fff p1 = dd2_mul(m, W[1]);
  fff t = dd2_add2(x0, p1.hi);
  float k1 = rint_(t.hi);
  fff s = dd2_add(t.hi - k1, t.lo + p1.lo);
  fff p2 = dd2_mul(m, W[2]);
  fff c = dd2_add2(s.hi, p2.hi);
  float lo = c.lo + (s.lo + (p2.lo + m * W[3]));
  j = (i0 - 4.0f * rint_(0.25f * i0)) + j0 + k1;
  return dd2_add(c.hi, lo);
}

constexpr float CWF_LIMIT = 65536.0f;

struct Trig32 {
  fff r;
  float j;
};

LMH_INLINE bool trigf_slow(float x) { return !(fabs_(x) < CWF_LIMIT); }
// |x| < 2^-12: sin x and tan x round to x, cos x to 1
LMH_INLINE bool trigf_tiny(float x) { return fabs_(x) < 0x1p-12f; }

LMH_INLINE Trig32 sincosf_fast(float x, bool is_cos) {
  float q, j;
  if (is_cos) {
    q = 2.0f * rint_(fma_(x, INV_PI_F, -0.5f)) + 1.0f;
    j = (q - 1.0f) * 0.5f + 1.0f;
  } else {
    q = rint_(x * INV_PI_F);
    j = q;
  }
  fff r = is_cos ? cwf_reduce<true>(x, q, PIH_F_C0, PIH_F_C1, PIH_F_C2, PIH_F_C3)
                 : cwf_reduce<false>(x, q, PI_F_C0, PI_F_C1, PI_F_C2, PI_F_C3);
  return Trig32{r, j};
}

LMH_INLINE Trig32 sincosf_slow(float x, bool is_cos) {
  // |x|/pi (+ 1/2 for cos) = j + f, as in the binary64 form
  float j;
  fff f = phf_core(fabs_(x), 1, is_cos ? 0.5f : 0.0f, j);
  fff r = dd2_mul(f, mk(2.0f * PIH2_F_H, 2.0f * PIH2_F_L));
  if (!is_cos && x < 0.0f) r = dd2_neg(r);
  r.hi = isfinite_(x) ? r.hi : __builtin_nanf("");
  return Trig32{r, j};
}

LMH_INLINE Trig32 sincosf_reduce(float x, bool is_cos) {
  Trig32 s;
  if (trigf_slow(x))
    s = sincosf_slow(x, is_cos);
  else
    s = sincosf_fast(x, is_cos);
  return s;
}

LMH_INLINE float sinf_poly_u10(fff r) {
  float z = r.hi * r.hi;
  float s3 = poly_estrin(z, SIN_S3_F32);
  fff r2 = dd2_squ(r);
  fff r3 = dd2_mul(r2, r);
  fff r5 = dd2_mul(r3, r2);
  fff c3 = dd2_mul(r3, mk(-SIXTH_F_H, -SIXTH_F_L));
  fff c5 = dd2_mul(r5, mk(INV120_F_H, INV120_F_L));
  float p7 = (r5.hi * z) * s3;
  fff s = dd2_add(r, c3);
  s = dd2_add(s, c5);
  return s.hi + (s.lo + p7);
}

LMH_INLINE float sinf_poly_u35(float r) {
  float z = r * r;
  return fma_(r * z, poly_estrin(z, SIN_S_F32), r);
}

LMH_INLINE float sinf_finish_u10(float x, Trig32 s) {
  float v = sinf_poly_u10(s.r);
  v = is_odd_intf(s.j) ? -v : v;
  return trigf_tiny(x) ? x : v;
}
LMH_INLINE float cosf_finish_u10(float x, Trig32 s) {
  float v = sinf_poly_u10(s.r);
  v = is_odd_intf(s.j) ? -v : v;
  return trigf_tiny(x) ? 1.0f : v;
}
LMH_INLINE float sinf_finish_u35(float x, Trig32 s) {
  float v = sinf_poly_u35(s.r.hi + s.r.lo);
  v = is_odd_intf(s.j) ? -v : v;
  return trigf_tiny(x) ? x : v;
}
LMH_INLINE float cosf_finish_u35(float x, Trig32 s) {
  float v = sinf_poly_u35(s.r.hi + s.r.lo);
  v = is_odd_intf(s.j) ? -v : v;
  return trigf_tiny(x) ? 1.0f : v;
}

// sincos in binary32: as the binary64 form
struct SinCos32 {
  Trig32 s, c;
};
LMH_INLINE SinCos32 sincosf2_fast(float x) {
  return SinCos32{sincosf_fast(x, false), sincosf_fast(x, true)};
}
LMH_INLINE Trig32 sincosf_raw(float x) { return sincosf_slow(x, false); }
LMH_INLINE SinCos32 sincosf_lift(float x, Trig32 raw) {
  return SinCos32{raw, sincosf_slow(x, true)};
}
LMH_INLINE SinCos32 sincosf2_reduce(float x) {
  SinCos32 s;
  if (trigf_slow(x))
    s = sincosf_lift(x, sincosf_raw(x));
  else
    s = sincosf2_fast(x);
  return s;
}

LMH_INLINE float sinf_u10(float x) { return sinf_finish_u10(x, sincosf_reduce(x, false)); }
LMH_INLINE float cosf_u10(float x) { return cosf_finish_u10(x, sincosf_reduce(x, true)); }
LMH_INLINE float sinf_u35(float x) { return sinf_finish_u35(x, sincosf_reduce(x, false)); }
LMH_INLINE float cosf_u35(float x) { return cosf_finish_u35(x, sincosf_reduce(x, true)); }

LMH_INLINE Trig32 tanf_fast(float x) {
  float k = rint_(x * TWO_OVER_PI_F);
  return Trig32{cwf_reduce<false>(x, k, PIH_F_C0, PIH_F_C1, PIH_F_C2, PIH_F_C3), k};
}

LMH_INLINE Trig32 tanf_slow(float x) {
  // x = j pi/2 + r with j modulo 4 (the bf16 finishers read the quadrant)
  float j;
  fff f = phf_core(fabs_(x), 0, 0.0f, j);
  fff r = dd2_mul(f, mk(PIH2_F_H, PIH2_F_L));
  if (x < 0.0f) {
    r = dd2_neg(r);
    j = -j;
  }
  r.hi = isfinite_(x) ? r.hi : __builtin_nanf("");
  return Trig32{r, j};
}

LMH_INLINE Trig32 tanf_reduce(float x) {
  Trig32 s;
  if (trigf_slow(x))
    s = tanf_slow(x);
  else
    s = tanf_fast(x);
  return s;
}

LMH_INLINE fff tanf_ff_finish(float x, Trig32 s) {
  fff y = dd2_scale(s.r, 0.5f);
  float z = y.hi * y.hi;
  float tp = poly_estrin(z, TAN_T_F32);
  fff y3 = dd2_mul(dd2_squ(y), y);
  fff t = dd2_add(y, dd2_mul(y3, tp));
  fff num = dd2_scale(t, 2.0f);
  fff den = dd2_add(1.0f, dd2_neg(dd2_squ(t)));
  if (is_odd_intf(s.j)) {
    fff tmp = num;
    num = den;
    den = dd2_neg(tmp);
  }
  fff q = dd2_div(num, den);
  return fabs_(x) < 0x1p-12f ? mk(x, 0.0f) : q;
}

LMH_INLINE fff tanf_ff(float x) { return tanf_ff_finish(x, tanf_reduce(x)); }

LMH_INLINE float tanf_finish_u10(float x, Trig32 s) {
  fff q = tanf_ff_finish(x, s);
  return trigf_tiny(x) ? x : q.hi + q.lo;
}

LMH_INLINE float tanf_finish_u35(float x, Trig32 s) {
  float y = (s.r.hi + s.r.lo) * 0.5f;
  float z = y * y;
  float t = fma_(y * z, poly_estrin(z, TAN_T_F32), y);
  float num = t + t;
  float den = fma_(-t, t, 1.0f);
  bool odd = is_odd_intf(s.j);
  float n2 = odd ? den : num;
  float d2 = odd ? -num : den;
  float res = n2 / d2;
  return trigf_tiny(x) ? x : res;
}

LMH_INLINE float tanf_u10(float x) { return tanf_finish_u10(x, tanf_reduce(x)); }
LMH_INLINE float tanf_u35(float x) { return tanf_finish_u35(x, tanf_reduce(x)); }

// ---------------------------------------------------------------------------
// pow, atan2
// ---------------------------------------------------------------------------
LMH_INLINE fff logf_ff(float a) {
  float e;
  fff t = logf_t(a, e);
  fff t2 = dd2_squ(t);
  float z = t2.hi;
  float rr = poly_estrin(z, LOG_R_F32);
  fff t3 = dd2_mul(t2, t);
  fff c3 = dd2_mul(t3, mk(TWOTHIRD_F_H, TWOTHIRD_F_L));
  float p5 = (t3.hi * z) * rr;
  fff l = dd2_add(dd2_scale(t, 2.0f), c3);
  l = dd2_add(l, p5);
  // e * LN2_HI_F is exact (16-bit head, |e| <= 150)
  fff el = mk(e * LN2_HI_F, e * LN2_LO_F);
  return dd2_add2(el, l);
}

// the Annex F values of pow around r = |x|^y (as in the binary64 form)
LMH_INLINE float powf_annexf(float x, float y, float r) {
  float ax = fabs_(x);
  bool yint = rint_(y) == y;
  bool yodd = fabs_(fma_(-2.0f, rint_(0.5f * y), y)) == 1.0f;
  bool xneg = __builtin_signbit(x);
  r = (xneg && yodd) ? -r : r;
  r = (x < 0.0f && !yint) ? __builtin_nanf("") : r;
  float mag = (ax == 0.0f) == (y < 0.0f) ? __builtin_inff() : 0.0f;
  r = (ax == 0.0f || isinf_(x)) ? ((xneg && yodd) ? -mag : mag) : r;
  float ymag = (ax < 1.0f) == (y < 0.0f) ? __builtin_inff() : 0.0f;
  r = isinf_(y) ? (ax == 1.0f ? 1.0f : ymag) : r;
  r = (isnan_(x) || isnan_(y)) ? __builtin_nanf("") : r;
  return (y == 0.0f || x == 1.0f) ? 1.0f : r;
}

// 3.5-ULP powf: the same float-float logarithm and product (the logarithm's
// relative error is multiplied by |y log x|, up to ~104), then the
// exponential in working precision: the reduced argument keeps the tail of
// the pair w, e^r = 1 + r + r^2 P(r) in binary32 (~1.3 ULP in all)
LMH_INLINE float expf_pair_ws(fff w, float& k) {
  float wh = w.hi > 104.0f ? 104.0f : (w.hi < -104.0f ? -104.0f : w.hi);
  float wl = wh == w.hi ? w.lo : 0.0f;
  k = rint_(wh * LOG2E_F);
  float r = fma_(k, -LN2_HI_F, wh) + (wl + k * -LN2_LO_F);
  return fma_(r * r, poly_estrin(r, EXP_P_F32), r) + 1.0f;
}

template <bool U10>
LMH_INLINE float powf_main(float x, float y, bool& rare) {
  float ax = fabs_(x);
  fff lg = logf_ff(ax);
  fff w = dd2_mul(lg, y);
  float k, r;
  if (U10) {
    fff e = expf_ff(w, k);
    r = ldexp_(e.hi + e.lo, (int)k);
  } else {
    float p = expf_pair_ws(w, k);
    r = ldexp_(p, (int)k);
  }
  // results below 2^-125; w clamped at -104 (e^w < 2^-150) rounds to zero
  rare = k <= -126.0f && w.hi >= -104.0f && isfinite_(ax) && ax != 0.0f && isfinite_(y);
  return powf_annexf(x, y, r);
}

// binary64 log and exp pairs (~2^-59 relative for |w| <= 104), one rounding
// at 2^-149; an exact tie between two subnormals is decided by ties-to-even
LMH_INLINE float powf_rare(float x, float y) {
  double axd = fabs_((double)x), yd = (double)y, kd, d;
  ddd ed = exp_dd(dd2_mul(log_dd(axd), yd), kd);
  double n = f32_sub_units(ed, (int)kd, d);
  if (fabs_(fabs_(d) - 0.5) < 0x1p-28) {
    double tie = pow_tie_units(axd, yd, 150.0);
    n = tie != 0.0 ? rint_(0.5 * tie) : n;
  }
  return powf_annexf(x, y, f32_from_units(n));
}

template <bool U10>
LMH_INLINE float powf_impl(float x, float y) {
  bool rare;
  float r = powf_main<U10>(x, y, rare);
  if (rare_lane(rare)) {
    float rs = powf_rare(rare ? x : 0.5f, rare ? y : 140.0f);
    r = rare ? rs : r;
  }
  return r;
}

LMH_INLINE float powf_u10(float x, float y) { return powf_impl<true>(x, y); }
LMH_INLINE float powf_u35(float x, float y) { return powf_impl<false>(x, y); }
LMH_INLINE float powf_u10_main(float x, float y, bool& rare) { return powf_main<true>(x, y, rare); }
LMH_INLINE float powf_u35_main(float x, float y, bool& rare) { return powf_main<false>(x, y, rare); }
LMH_INLINE float powf_u10_rare(float x, float y) { return powf_rare(x, y); }
LMH_INLINE float powf_u35_rare(float x, float y) { return powf_rare(x, y); }

// binary32 forms of atan_poly / atan_ratio (the extra reduction above
// tan(pi/8) through pi/4 + atan((n - d)/(n + d)))
constexpr float TAN_PI8_F = 0x1.a82798p-2f;           // tan(pi/8), rounded down
LMH_INLINE fff atanf_poly(fff v) {
  float z = v.hi * v.hi;
  float b2 = poly_estrin(z, ATAN_B2_F32);
  fff v3 = dd2_mul(dd2_squ(v), v);
  fff c3 = dd2_mul(v3, mk(-THIRD_F_H, -THIRD_F_L));
  float p5 = (v3.hi * z) * b2;
  return dd2_add(dd2_add(v, c3), p5);
}

LMH_INLINE fff atanf_ratio(float n, float d, fff& q, bool& red) {
  red = n > TAN_PI8_F * d;
  fff num = red ? dd2_add2(n, -d) : mk(n, 0.0f);
  fff den = red ? dd2_add2(n, d) : mk(d, 0.0f);
  q = dd2_div(num, den);
  fff a = atanf_poly(red ? dd2_neg(q) : q);
  return red ? dd2_add(mk(0.5f * PIH2_F_H, 0.5f * PIH2_F_L), dd2_neg(a)) : a;
}

LMH_INLINE float atan2f_u10(float y, float x) {
  float ay = fabs_(y), ax = fabs_(x);
  bool both_inf = isinf_(ax) && isinf_(ay);
  ay = both_inf ? 1.0f : ay;
  ax = both_inf ? 1.0f : ax;
  bool swap = ay > ax;
  float n = swap ? ax : ay;
  float d = swap ? ay : ax;
  int de = frexp_exp_(d);
  float dn = ldexp_(d, -de);
  float nn = ldexp_(n, -de);
  fff t;
  bool red;
  fff a = atanf_ratio(nn, dn, t, red);
  t = isinf_(d) ? mk(0.0f, 0.0f) : t;
  a = isinf_(d) ? mk(0.0f, 0.0f) : a;
  if (!red && t.hi < 0x1p-100f) {                           // see atan2_u10
    float q = n / d;
    float r = fma_(-ldexp_(q, 60), d, ldexp_(n, 60));
    bool tie_up = r < 0.0f && -r == ldexp_(d, -90);
    a = mk(tie_up ? pred_(q) : q, 0.0f);
  }
  if (swap) a = dd2_add(mk(PIH2_F_H, PIH2_F_L), dd2_neg(a));
  bool xneg = __builtin_signbit(x);
  if (xneg) a = dd2_add(mk(PI2_F_H, PI2_F_L), dd2_neg(a));
  float r = copysign_(a.hi + a.lo, y);
  if (y == 0.0f) r = xneg ? copysign_(PI2_F_H, y) : copysign_(0.0f, y);
  r = (isnan_(x) || isnan_(y)) ? __builtin_nanf("") : r;
  return r;
}

// ---------------------------------------------------------------------------
// atan, asin, acos in binary32: the binary64 methods with float-float pairs
// ---------------------------------------------------------------------------
LMH_INLINE float atanf_u10(float x) {
  float ax = fabs_(x);
  bool big = ax > 1.0f;
  fff t;
  bool red;
  fff a = atanf_ratio(big ? 1.0f : ax, big ? ax : 1.0f, t, red);
  a = isinf_(ax) ? mk(0.0f, 0.0f) : a;
  if (big) a = dd2_add(mk(PIH2_F_H, PIH2_F_L), dd2_neg(a));
  return copysign_(a.hi + a.lo, x);
}

LMH_INLINE float atanf_u35(float x) {
  float ax = fabs_(x);
  bool big = ax > 1.0f;
  float t = big ? 1.0f / ax : ax;
  float z = t * t;
  float p = fma_(t * z, poly_estrin(z, ATAN_A_F32), t);
  float r = big ? (PIH2_F_H - p) + PIH2_F_L : p;
  return copysign_(r, x);
}

LMH_INLINE fff asinf_poly(fff s) {
  float z = s.hi * s.hi;
  float t = (s.hi * z) * poly_estrin(z, ASIN_S_F32);
  return dd2_add(s, t);
}

LMH_INLINE fff asinf_reduce(float ax, bool exact_root) {
  float z = (1.0f - ax) * 0.5f;
  float sh = __builtin_sqrtf(z);
  float e = fma_(-sh, sh, z);
  float sl = (exact_root && z > 0.0f) ? e / (sh + sh) : 0.0f;
  return mk(sh, sl);
}

template <bool U10>
LMH_INLINE fff asinf_abs(float ax, bool& reduced) {
  reduced = ax > 0.5f;
  fff s = reduced ? asinf_reduce(ax, U10) : mk(ax, 0.0f);
  return asinf_poly(s);
}

template <bool U10>
LMH_INLINE float asinf_impl(float x) {
  float ax = fabs_(x);
  bool red;
  fff a = asinf_abs<U10>(ax, red);
  if (red) a = dd2_add(mk(PIH2_F_H, PIH2_F_L), dd2_scale(a, -2.0f));
  float r = copysign_(a.hi + a.lo, x);
  return ax > 1.0f ? __builtin_nanf("") : r;
}

template <bool U10>
LMH_INLINE float acosf_impl(float x) {
  float ax = fabs_(x);
  bool red;
  fff a = asinf_abs<U10>(ax, red);
  bool neg = x < 0.0f;
  fff r;
  if (red) {
    a = dd2_scale(a, 2.0f);
    r = neg ? dd2_add(mk(PI2_F_H, PI2_F_L), dd2_neg(a)) : a;
  } else {
    a = neg ? dd2_neg(a) : a;
    r = dd2_add(mk(PIH2_F_H, PIH2_F_L), dd2_neg(a));
  }
  float v = r.hi + r.lo;
  return (ax > 1.0f || isnan_(x)) ? __builtin_nanf("") : v;
}

LMH_INLINE float asinf_u10(float x) { return asinf_impl<true>(x); }
LMH_INLINE float asinf_u35(float x) { return asinf_impl<false>(x); }
LMH_INLINE float acosf_u10(float x) { return acosf_impl<true>(x); }
LMH_INLINE float acosf_u35(float x) { return acosf_impl<false>(x); }

// ---------------------------------------------------------------------------
// hyperbolic functions
// ---------------------------------------------------------------------------
LMH_INLINE fff expf_half(float ax, float& k) {   // e^ax / 2
  fff w = dd2_add2(ax, -LN2_F_H);
  w.lo += -LN2_F_L;
  return expf_ff(dd2_norm(w), k);
}

LMH_INLINE float sinhf_u10(float x) {
  float ax = fabs_(x);
  float r;
  if (ax < 1.0f) {
    float z = x * x;
    r = fma_(x * z, poly_estrin(z, SINH_H_F32), x);
  } else {
    float k;
    fff e = expf_half(ax > 90.0f ? 90.0f : ax, k);
    fff h = mk(ldexp_(e.hi, (int)k), ldexp_(e.lo, (int)k));
    fff rc = dd2_rec(e);
    fff g = mk(ldexp_(rc.hi, -(int)k - 2), ldexp_(rc.lo, -(int)k - 2));
    fff s = dd2_add(h, dd2_neg(g));
    r = s.hi + s.lo;
    r = isinf_(h.hi) ? __builtin_inff() : r;
    r = copysign_(r, x);
  }
  return isnan_(x) ? x : r;
}

LMH_INLINE float coshf_u10(float x) {
  float ax = fabs_(x);
  float k;
  fff e = expf_half(ax > 90.0f ? 90.0f : ax, k);
  fff h = mk(ldexp_(e.hi, (int)k), ldexp_(e.lo, (int)k));
  fff rc = dd2_rec(e);
  fff g = mk(ldexp_(rc.hi, -(int)k - 2), ldexp_(rc.lo, -(int)k - 2));
  fff s = dd2_add(h, g);
  float r = s.hi + s.lo;
  r = isinf_(h.hi) ? __builtin_inff() : r;
  return isnan_(x) ? x : r;
}

LMH_INLINE float tanhf_u10(float x) {
  float ax = fabs_(x);
  float r;
  if (ax < 0.625f) {
    float z = x * x;
    r = fma_(x * z, poly_estrin(z, TANH_G_F32), x);
  } else {
    float a2 = ax > 20.0f ? 40.0f : ax + ax;
    float k;
    fff e = expf_ff(mk(a2, 0.0f), k);
    fff E = mk(ldexp_(e.hi, (int)k), ldexp_(e.lo, (int)k));
    fff den = dd2_add(E, 1.0f);
    fff q = dd2_div(mk(2.0f, 0.0f), den);
    fff s = dd2_add(1.0f, dd2_neg(q));
    r = copysign_(s.hi + s.lo, x);
  }
  r = fabs_(x) < 0x1p-12f ? x : r;
  return isnan_(x) ? x : r;
}

// ---------------------------------------------------------------------------
// 3.5-ULP atan2, sinh, cosh, tanh in binary32 (the binary64 forms' structure)
// ---------------------------------------------------------------------------
LMH_INLINE float atan2f_u35_finish(float y, float x, float a, bool swap) {
  a = swap ? (PIH2_F_H - a) + PIH2_F_L : a;
  bool xneg = __builtin_signbit(x);
  a = xneg ? (PI2_F_H - a) + PI2_F_L : a;
  float r = copysign_(a, y);
  if (y == 0.0f) r = xneg ? copysign_(PI2_F_H, y) : copysign_(0.0f, y);
  return (isnan_(x) || isnan_(y)) ? __builtin_nanf("") : r;
}

LMH_INLINE float atan2f_u35_main(float y, float x, bool& rare) {
  float ay = fabs_(y), ax = fabs_(x);
  bool both_inf = isinf_(ax) && isinf_(ay);
  ay = both_inf ? 1.0f : ay;
  ax = both_inf ? 1.0f : ax;
  bool swap = ay > ax;
  float t = (swap ? ax : ay) / (swap ? ay : ax);
  float z = t * t;
  float a = fma_(t * z, poly_estrin(z, ATAN_A_F32), t);
  rare = !swap && t < 0x1p-100f && t != 0.0f;
  return atan2f_u35_finish(y, x, a, swap);
}

LMH_INLINE float atan2f_u35_rare(float y, float x) {   // see atan2_u35_rare
  float n = fabs_(y), d = fabs_(x);
  float t = n / d;
  float r0 = fma_(-ldexp_(t, 60), d, ldexp_(n, 60));
  float a = (r0 < 0.0f && -r0 == ldexp_(d, -90)) ? pred_(t) : t;
  return atan2f_u35_finish(y, x, a, false);
}

LMH_INLINE float atan2f_u35(float y, float x) {
  bool rare;
  float r = atan2f_u35_main(y, x, rare);
  if (rare_lane(rare)) {
    float rs = atan2f_u35_rare(rare ? y : 1.0f, rare ? x : 2.0f);
    r = rare ? rs : r;
  }
  return r;
}

// e^a 2^-s in working precision (|a| <= 104 keeps k * LN2_HI exact)
LMH_INLINE float expf_ws(float a, int s) {
  float k = rint_(a * LOG2E_F);
  float s0 = fma_(k, -LN2_HI_F, a);
  float t = k * -LN2_LO_F;
  float rh = s0 + t;
  float rl = (s0 - rh) + t;
  fff e = expf_core(rh, rl);
  return ldexp_(e.hi + e.lo, (int)k - s);
}

LMH_INLINE float sinhf_u35(float x) {
  float ax = fabs_(x);
  float r;
  if (ax < 1.0f) {
    float z = x * x;
    r = fma_(x * z, poly_estrin(z, SINH_H_F32), x);
  } else {
    float e = expf_ws(ax > 90.0f ? 90.0f : ax, 1);
    r = copysign_(e - 0.25f / e, x);
  }
  return isnan_(x) ? x : r;
}

LMH_INLINE float coshf_u35(float x) {
  float ax = fabs_(x);
  float e = expf_ws(ax > 90.0f ? 90.0f : ax, 1);
  float r = e + 0.25f / e;
  return isnan_(x) ? x : r;
}

LMH_INLINE float tanhf_u35(float x) {
  float ax = fabs_(x);
  float r;
  if (ax < 0.625f) {
    float z = x * x;
    r = fma_(x * z, poly_estrin(z, TANH_G_F32), x);
  } else {
    float e2 = expf_ws(ax > 20.0f ? 40.0f : ax + ax, 0);
    r = copysign_(1.0f - 2.0f / (e2 + 1.0f), x);
  }
  r = ax < 0x1p-12f ? x : r;                       // keeps tanh(-0) = -0
  return isnan_(x) ? x : r;
}

// ---------------------------------------------------------------------------
// log10, log1p, exp10, expm1, cbrt, hypot in binary32 (the binary64 forms'
// structure)
// ---------------------------------------------------------------------------
LMH_INLINE fff logf_pair(fff t, float e) {
  float z = t.hi * t.hi;
  float t3q = (t.hi * z) * poly_estrin(z, LOG_Q_F32);
  fff lm = dd2_add(t.hi + t.hi, (t.lo + t.lo) + t3q);
  fff s = dd2_add2(e * LN2_HI_F, lm.hi);            // e*LN2_HI is exact
  return mk(s.hi, s.lo + (lm.lo + e * LN2_LO_F));
}

LMH_INLINE float logf_specials(float x, float r) {
  r = x == 0.0f ? -__builtin_inff() : r;
  r = x < 0.0f ? __builtin_nanf("") : r;
  return (isinf_(x) && x > 0.0f) || isnan_(x) ? x : r;
}

LMH_INLINE float log10f_u10(float x) {
  float e;
  fff t = logf_t(x, e);
  fff l = dd2_mul(dd2_norm(logf_pair(t, e)), mk(INVLN10_F_H, INVLN10_F_L));
  return logf_specials(x, l.hi + l.lo);
}

LMH_INLINE float log1pf_u10(float x) {
  fff a = dd2_add2(1.0f, x);
  float m = frexp_mant_(a.hi);
  int ie = frexp_exp_(a.hi);
  ie = m < 0.75f ? ie - 1 : ie;
  float mh = ldexp_(a.hi, -ie), ml = ldexp_(a.lo, -ie);
  fff num = dd2_add2(mh - 1.0f, ml);
  fff den = dd2_add(dd2_add(1.0f, mh), ml);
  fff l = logf_pair(dd2_div(num, den), (float)ie);
  float r = l.hi + l.lo;
  r = x == -1.0f ? -__builtin_inff() : r;
  r = x < -1.0f ? __builtin_nanf("") : r;
  r = (isinf_(x) && x > 0.0f) || isnan_(x) ? x : r;
  return fabs_(x) < 0x1p-25f ? x : r;               // rounds to x; keeps +-0
}

// |x| <= 50 covers every finite, nonzero binary32 result; |k| <= 167 keeps
// k * LN2_HI (16 bits) exact
LMH_INLINE float exp10f_u10_main(float x, bool& rare) {
  float xc = x > 50.0f ? 50.0f : (x < -50.0f ? -50.0f : x);
  float k = rint_(xc * LOG2_10_F);
  fff a = dd2_mul(xc, LN10_F_H);
  float s = fma_(k, -LN2_HI_F, a.hi);
  float t = fma_(xc, LN10_F_L, a.lo) + k * -LN2_LO_F;
  fff r = dd2_add2(s, t);
  fff e = expf_core(r.hi, r.lo);
  rare = k <= -126.0f && k >= -151.0f;              // the clamp gives k = -166
  float v = ldexp_(e.hi + e.lo, (int)k);
  return isnan_(x) ? x : v;
}

// binary64: x ln10 as an exact pair plus x times ln10's tail
LMH_INLINE float exp10f_u10_rare(float x) {        // -45.5 < x < -37.7
  double xd = (double)x, d;
  double kd = rint_(xd * LOG2_10_D);
  ddd a = dd2_mul(xd, LN10_D_H);
  ddd rd = dd2_add2(fma_(kd, -LN2_HI_D, a.hi), fma_(xd, LN10_D_L, a.lo) + kd * -LN2_LO_D);
  return f32_from_units(f32_sub_units(exp_core(rd.hi, rd.lo), (int)kd, d));
}

LMH_INLINE float exp10f_u10(float x) {
  bool rare;
  float r = exp10f_u10_main(x, rare);
  if (rare_lane(rare)) {
    float rs = exp10f_u10_rare(rare ? x : -40.0f);
    r = rare ? rs : r;
  }
  return r;
}

// below -18, e^x is under half an ulp of 1 (2^-25) and the result is -1
LMH_INLINE float expm1f_u10(float x) {
  float xc = x > 89.0f ? 89.0f : (x < -18.0f ? -18.0f : x);
  float k = rint_(xc * LOG2E_F);
  float s0 = fma_(k, -LN2_HI_F, xc);
  float t0 = k * -LN2_LO_F;
  float rh = s0 + t0;
  float rl = (s0 - rh) + t0;
  fff h = dd2_mul(rh, rh);
  fff em = dd2_add(rh, mk(0.5f * h.hi, 0.5f * h.lo));
  em.lo += fma_(rh * h.hi, poly_estrin_tail<1>(rh, EXP_P_F32), fma_(rh, rl, rl));
  int kh = (int)k - 1;
  fff t = mk(ldexp_(em.hi, kh), ldexp_(em.lo, kh));
  fff d = dd2_add2(ldexp_(1.0f, kh), -0.5f);
  fff sum = dd2_add2(t, d);
  float r = 2.0f * (sum.hi + sum.lo);
  r = x < -18.0f ? -1.0f : r;
  r = isnan_(x) ? x : r;
  return fabs_(x) < 0x1p-25f ? x : r;
}

// asinh, acosh, atanh in float-float, the binary64 forms' structure:
// log1p of an argument formed without cancellation, sqrt from the
// reciprocal square root estimate, one Newton step and the pair's residual,
// log1p(u) = log((1 + u) 2^-e) + e ln2 from the float-float log pair.
// Above 2^60 (where x^2 would near binary32's range) asinh and acosh take
// log1p(|x|) + ln2 (the omitted 1/(4 x^2) is below 2^-120).
LMH_INLINE fff sqrtf_ff(fff p) {
  float g = rsq_(p.hi);
  float h = 0.5f * g;
  float r = p.hi * g;
  r = fma_(h, fma_(-r, r, p.hi), r);
  fff q = dd2_mul(r, r);
  float res = ((p.hi - q.hi) - q.lo) + p.lo;
  return dd2_add(r, res * h);
}

LMH_INLINE fff log1pf_ff(fff u) {                   // u > -1
  fff a = dd2_add2(1.0f, u.hi);
  a.lo += u.lo;
  float m = frexp_mant_(a.hi);
  int ie = frexp_exp_(a.hi);
  ie = m < 0.75f ? ie - 1 : ie;
  float mh = ldexp_(a.hi, -ie), ml = ldexp_(a.lo, -ie);
  fff num = dd2_add2(mh - 1.0f, ml);                 // mh - 1 is exact
  fff den = dd2_add(dd2_add(1.0f, mh), ml);
  return logf_pair(dd2_div(num, den), (float)ie);
}

constexpr float INVHYP_BIG_F = 0x1p60f;

LMH_INLINE float asinhf_u10(float x) {
  float ax = fabs_(x);
  bool big = ax > INVHYP_BIG_F;
  float a = big ? 1.0f : ax;
  fff x2 = dd2_mul(a, a);
  fff den = dd2_add(sqrtf_ff(dd2_add2(x2, 1.0f)), 1.0f);
  fff u = dd2_add(a, dd2_div(x2, den));
  fff l = log1pf_ff(big ? mk(ax, 0.0f) : u);
  l = dd2_add(l, big ? mk(LN2_F_H, LN2_F_L) : mk(0.0f, 0.0f));
  float r = copysign_(l.hi + l.lo, x);
  r = ax < 0x1p-12f || isinf_(x) ? x : r;            // asinh x rounds to x; +-inf
  return isnan_(x) ? x : r;
}

LMH_INLINE float acoshf_u10(float x) {
  bool big = x > INVHYP_BIG_F;
  float a = big ? 2.0f : x;
  fff d = dd2_add2(a, -1.0f);
  fff u = dd2_add(sqrtf_ff(dd2_mul(d, dd2_add2(a, 1.0f))), d);
  fff l = log1pf_ff(big ? mk(x, 0.0f) : u);
  l = dd2_add(l, big ? mk(LN2_F_H, LN2_F_L) : mk(0.0f, 0.0f));
  float r = l.hi + l.lo;
  r = x == 1.0f ? 0.0f : r;
  r = x < 1.0f ? __builtin_nanf("") : r;
  return isinf_(x) && x > 0.0f ? x : (isnan_(x) ? x : r);
}

LMH_INLINE float atanhf_u10(float x) {
  float ax = fabs_(x);
  fff u = dd2_div(mk(2.0f * ax, 0.0f), dd2_add2(1.0f, -ax));
  fff l = log1pf_ff(u);
  float r = copysign_(0.5f * (l.hi + l.lo), x);
  r = ax == 1.0f ? copysign_(__builtin_inff(), x) : r;
  r = ax > 1.0f ? __builtin_nanf("") : r;
  r = ax < 0x1p-12f ? x : r;                         // atanh x rounds to x
  return isnan_(x) ? x : r;
}

// erf, erfc in float-float, the binary64 forms' structure: |x| < 0.75:
// erf x = c0 x + c1 x^3 + x^5 P(x^2) with c0 = 2/sqrt(pi) and c1 = -c0/3 as
// pairs; 0.75 <= |x| < 10.1: erfc |x| = e^(-x^2) g(|x|) with g from the
// binary32 rows of the generated table (fitted to 2^-30; constant and linear
// coefficients as pairs), e^(-x^2) from the
// exact square through the float-float exp, erf = 1 - erfc below 4 and
// erfc(-|x|) = 2 - erfc|x|.  Results in or near the subnormal range take
// binary64 rare paths (erfc above 9.1; erf below 2^-100, where c0 x must be
// rounded from an exact product).
constexpr float ERFF_SMALL = 0.75f;

LMH_INLINE fff erff_small(float x) {                  // |x| < 0.75
  fff x3 = dd2_mul(dd2_mul(x, x), x);
  float z = x * x;
  fff v = dd2_add(dd2_mul(mk(TWO_OVER_SQRTPI_F_H, TWO_OVER_SQRTPI_F_L), x),
                  dd2_mul(x3, mk(ERF_C1_F_H, ERF_C1_F_L)));
  return mk(v.hi, v.lo + (x3.hi * z) * poly_estrin(z, ERF_P_F32));
}

LMH_INLINE fff erfcf_poly(float a, bool& inv) {
  int row = (a >= 1.0f) + (a >= 1.5f) + (a >= 2.25f) + (a >= 3.5f) + (a >= 6.0f);
  inv = row >= 3;
  float s = (inv ? rcp_refined(a) : a) - ERFCF_C[row];
  const float* P = ERFCF_TAB + row;                  // column-major: entry k at P[k * ROWS]
  float q[ERFCF_TERMS - 2];
#pragma unroll
  for (int i = 0; i < ERFCF_TERMS - 2; ++i) q[i] = P[(4 + i) * ERFCF_ROWS];
  // g = c0 + s (c1 + s Q(s)), c0 and c1 as pairs: the linear term reaches
  // about a third of g, so its product stays a pair
  fff u = dd2_add(mk(P[2 * ERFCF_ROWS], P[3 * ERFCF_ROWS]), s * poly_estrin(s, q));
  return dd2_add(mk(P[0], P[ERFCF_ROWS]), dd2_mul(u, s));
}

// erfc(a) = pair * 2^k for 0.75 <= a < 10.1
LMH_INLINE fff erfcf_big(float a, float& k) {
  bool inv;
  fff g = erfcf_poly(a, inv);
  fff x2 = dd2_mul(a, a);
  fff e = expf_ff(mk(-x2.hi, -x2.lo), k);
  fff r = dd2_mul(e, g);
  return inv ? dd2_div(r, mk(a, 0.0f)) : r;
}

LMH_INLINE float erff_u10_main(float x, bool& rare) {
  float a = fabs_(x);
  fff sm = erff_small(a < ERFF_SMALL ? x : 0.0f);
  float r = sm.hi + sm.lo;
  bool mid = a >= ERFF_SMALL && a < 4.0f;             // above 4 erf rounds to +-1
  if (any_lane(mid)) {
    float k;
    fff e = erfcf_big(mid ? a : 1.0f, k);
    fff d = dd2_add(1.0f, mk(-ldexp_(e.hi, (int)k), -ldexp_(e.lo, (int)k)));
    float v = copysign_(d.hi + d.lo, x);
    r = mid ? v : r;
  }
  r = a >= 4.0f ? copysign_(1.0f, x) : r;
  rare = a < 0x1p-100f && a != 0.0f;
  return isnan_(x) || x == 0.0f ? x : r;              // keeps erf(-0) = -0
}

// erf x = c0 x below 2^-100 (the next term is 2^-200 smaller), where the
// float pair's low word would fall below the normal range: subnormal
// results (|x| < 2^-125) from the exact binary64 product pair of c0 and
// x 2^149 rounded once to units of 2^-149, the others from the binary64
// product rounded to binary32
LMH_INLINE float erff_u10_rare(float x) {
  double d;
  ddd v = dd2_mul(mk(TWO_OVER_SQRTPI_D_H, TWO_OVER_SQRTPI_D_L), ldexp_((double)x, 149));
  float sub = f32_from_units(f32_sub_units(v, -149, d));
  float nrm = (float)(TWO_OVER_SQRTPI_D_H * (double)x);
  return fabs_(x) < 0x1p-125f ? sub : nrm;
}

LMH_INLINE float erff_u10(float x) {
  bool rare;
  float r = erff_u10_main(x, rare);
  if (rare_lane(rare)) {
    float rs = erff_u10_rare(rare ? x : 0.0f);
    r = rare ? rs : r;
  }
  return r;
}

LMH_INLINE float erfcf_u10_main(float x, bool& rare) {
  float a = fabs_(x);
  fff sm = erff_small(a < ERFF_SMALL ? x : 0.0f);
  fff one_m = dd2_add(1.0f, mk(-sm.hi, -sm.lo));
  float r = one_m.hi + one_m.lo;
  bool tab = a >= ERFF_SMALL && a < 10.1f;            // erfc(10.1) < 2^-150
  if (any_lane(tab)) {
    float k;
    fff e = erfcf_big(tab ? a : 1.0f, k);
    float pos = ldexp_(e.hi + e.lo, (int)k);
    fff two_m = dd2_add(2.0f, mk(-ldexp_(e.hi, (int)k), -ldexp_(e.lo, (int)k)));
    float v = x > 0.0f ? pos : two_m.hi + two_m.lo;
    r = tab ? v : r;
  }
  r = x >= 10.1f ? 0.0f : r;
  r = x <= -10.1f ? 2.0f : r;
  rare = x > 9.1f && x < 10.1f;                       // results near or below 2^-126
  return isnan_(x) ? x : r;
}

// binary32 erfc above 9.1 (results near or in the subnormal range): the
// binary64 polynomials and exp in working precision, rounded once
LMH_INLINE float erfcf_u10_rare(float x) {
  double a = (double)x;
  bool inv;
  ddd g = erfc_poly(a, inv);
  double v = exp_ws(-(a * a), 0) * (g.hi + g.lo);
  return (float)(inv ? v / a : v);
}

LMH_INLINE float erfcf_u10(float x) {
  bool rare;
  float r = erfcf_u10_main(x, rare);
  if (rare_lane(rare)) {
    float rs = erfcf_u10_rare(rare ? x : 9.5f);
    r = rare ? rs : r;
  }
  return r;
}

// cbrt in float-float: |x| = a 2^(3q) with a = m 2^i in [0.5, 4); y0 = a z^2
// from the seed z ~ a^(-1/3) (about 2^-21), then one Newton step on
// y^3 = a with the residual a - y0^3 from exact products (y0^2 = P + p,
// y0 P = T + t; a - T is exact, T being within a factor two of a) and
// 1/(3 y0^2) taken as z^2 / 3: about 2^-42 before the one rounding in the
// last FMA.  A binary32 cube root is never a midpoint (its cube would need
// 73 bits) nor subnormal (|x| >= 2^-149 gives at least 2^-49.7).
LMH_INLINE float cbrtf_u10(float x) {
  float ax = fabs_(x);
  float m = frexp_mant_(ax);
  int e = frexp_exp_(ax);
  int q = (e + 300) / 3 - 100;                       // floor(e / 3)
  float a = ldexp_(m, e - 3 * q);
  float z = rcbrt_seed(a);
  float z2 = z * z;
  float y0 = a * z2;
  fff p = dd2_mul(y0, y0);
  fff t = dd2_mul(y0, p.hi);
  float d = ((a - t.hi) - t.lo) - y0 * p.lo;
  float r = ldexp_(fma_(d * (1.0f / 3.0f), z2, y0), q);
  r = copysign_(r, x);
  return (x == 0.0f || !isfinite_(x)) ? x : r;
}

// hypot: |x|, |y| scaled by 2^-s (s the larger one's exponent), the sum of
// squares as a float-float pair (exact products, one fast two-sum), its
// square root from the reciprocal square root estimate, one Newton step
// and a correction by the pair's residual (about 2^-46), rounded once.
// Subnormal results (s <= -125) need more: sqrt(N) 2^-149 for an integer
// N < 2^48 comes within 2^-26.5 units of a rounding midpoint, which 2^-46
// relative does not resolve, so those lanes take the rare path, where N is
// exact in binary64 and its correctly rounded square root decides.
LMH_INLINE float hypotf_u10_main(float x, float y, bool& rare) {
  float ax = fabs_(x), ay = fabs_(y);
  float n = ax > ay ? ax : ay, d = ax > ay ? ay : ax;
  int s = frexp_exp_(n);
  float ns = ldexp_(n, -s), ds = ldexp_(d, -s);
  fff S = dd2_add(dd2_mul(ns, ns), dd2_mul(ds, ds));
  float g = rsq_(S.hi);
  float h = 0.5f * g;
  float r = S.hi * g;
  r = fma_(h, fma_(-r, r, S.hi), r);
  fff p = dd2_mul(r, r);
  float res = ((S.hi - p.hi) - p.lo) + S.lo;
  float v = ldexp_(fma_(res, h, r), s);
  rare = s <= -125 && n != 0.0f;
  v = n == 0.0f ? 0.0f : v;
  v = isnan_(x) || isnan_(y) ? __builtin_nanf("") : v;
  return isinf_(x) || isinf_(y) ? __builtin_inff() : v;
}

LMH_INLINE float hypotf_u10_rare(float x, float y) {     // |x|, |y| < 2^-125
  double a = (double)x, b = (double)y;
  return (float)__builtin_sqrt(fma_(a, a, b * b));
}

LMH_INLINE float hypotf_u10(float x, float y) {
  bool rare;
  float r = hypotf_u10_main(x, y, rare);
  if (rare_lane(rare)) {
    float rs = hypotf_u10_rare(rare ? x : 0.0f, rare ? y : 0.0f);
    r = rare ? rs : r;
  }
  return r;
}

// ---------------------------------------------------------------------------
// exact remainders in binary32 (same long division as binary64)
// ---------------------------------------------------------------------------

// lgamma and tgamma in binary32: the binary64 evaluators' pairs rounded once
// into binary32 (lgamma never has a binary32 subnormal result; tgamma's
// subnormal results are rounded from the exponential's pair at 2^-149).
LMH_INLINE float lgammaf_u10(float x) {
  double r = lgamma_u10((double)x);
  return (float)r;
}

LMH_INLINE float tgammaf_u10_main(float x, bool& rare) {
  bool rare64;                       // binary64 subnormal results: zero in binary32
  float r = (float)tgamma_u10_main((double)x, rare64);
  rare = fabs_(r) < 0x1p-125f && isfinite_(x) && x < 0.0f && rint_(x) != x && x > -60.0f;
  return r;
}

LMH_INLINE float tgammaf_u10_rare(float x) {       // results below 2^-125
  double xd = (double)x, k, d;
  bool ovf;
  ddd l = lgamma_dd<false>(xd, ovf);
  ddd e = exp_dd(l, k);
  float v = f32_from_units(f32_sub_units(e, (int)k, d));
  return floor_is_odd(xd) ? -v : v;
}

LMH_INLINE float tgammaf_u10(float x) {
  bool rare;
  float r = tgammaf_u10_main(x, rare);
  if (rare_lane(rare)) {
    float rs = tgammaf_u10_rare(rare ? x : -40.5f);
    r = rare ? rs : r;
  }
  return r;
}

LMH_INLINE fff fmodf_step(fff r, float d, float dm, float rdm, int de) {   // see fmod_step
  float rm = frexp_mant_(r.hi);
  int re = frexp_exp_(r.hi);
  int E = re - de;
  float qf = pred_(rm) * rdm;
  float qs = E < 25 ? ldexp_(trunc_(ldexp_(qf, E)), -E) : qf;
  qs = (r.hi < 3.0f * d && r.hi > d) ? ldexp_(2.0f, -E) : qs;
  qs = (r.hi < 2.0f * d && r.hi > d) ? ldexp_(1.0f, -E) : qs;
  qs = r.hi == d ? (r.lo >= 0.0f ? ldexp_(1.0f, -E) : 0.0f) : qs;
  fff p = dd2_mul(qs, dm);
  p = mk(ldexp_(p.hi, re), ldexp_(p.lo, re));
  return dd2_norm(dd2_add2(r, dd2_neg(p)));
}

LMH_INLINE float fmodf_core_steps(float n, float d, int& steps) {   // see fmod_core_steps
  float dm = frexp_mant_(d);
  int de = frexp_exp_(d);
  float rdm = pred_(1.0f / dm);
  fff r = mk(n, 0.0f);
  bool active = r.hi > d || (r.hi == d && r.lo >= 0.0f);
  steps = 0;
  for (int it = 0; it < 64 && any_lane(active); ++it) {
    if (active) {
      ++steps;
      r = fmodf_step(r, d, dm, rdm, de);
      active = r.hi > d || (r.hi == d && r.lo >= 0.0f);
    }
  }
  return r.hi;
}

LMH_INLINE float fmodf_core(float n, float d) {
  int steps;
  return fmodf_core_steps(n, d, steps);
}

LMH_INLINE float fmodf_f32(float x, float y) {
  float n = fabs_(x), d = fabs_(y);
  bool special = !isfinite_(x) || !isfinite_(d) || d == 0.0f || n < d;
  float r = fmodf_core(special ? 0.0f : n, special ? 1.0f : d);
  r = copysign_(r, x);
  r = n < d ? x : r;
  r = isinf_(d) && isfinite_(x) ? x : r;
  r = (d == 0.0f || !isfinite_(x) || isnan_(y)) ? __builtin_nanf("") : r;
  return r;
}

LMH_INLINE float remainderf_f32(float x, float y) {
  float n = fabs_(x), d = fabs_(y);
  float d2 = d + d;
  bool special = !isfinite_(x) || !isfinite_(d) || d == 0.0f;
  bool small = n < d2;
  float r2 = fmodf_core(special || small ? 0.0f : n, special || small ? 1.0f : d2);
  r2 = small ? n : r2;
  bool odd = r2 >= d;
  float r1 = odd ? r2 - d : r2;
  float tw = r1 + r1;
  r1 = (tw > d || (tw == d && odd)) ? r1 - d : r1;
  float r = r1 * copysign_(1.0f, x);
  r = isinf_(d) && isfinite_(x) ? x : r;
  r = (d == 0.0f || !isfinite_(x) || isnan_(y)) ? __builtin_nanf("") : r;
  return r;
}

// fdim, fmax, fmin (C99 functions of the paper's set, Section 1, shown there
// only as a masking example): fdim(x, y) = x - y (one rounding) when x > y,
// else +0, NaN if either is NaN; fmax / fmin pick the larger / smaller
// argument, the other one when one is NaN, with -0 ordered below +0
LMH_INLINE float fdimf_f32(float x, float y) {
  float d = x > y ? x - y : 0.0f;
  return (isnan_(x) || isnan_(y)) ? __builtin_nanf("") : d;
}
LMH_INLINE float fmaxf_f32(float x, float y) {
  bool zeros = x == 0.0f && y == 0.0f;
  float r = (x > y || isnan_(y)) ? x : y;
  return zeros ? (__builtin_signbit(x) ? y : x) : r;
}
LMH_INLINE float fminf_f32(float x, float y) {
  bool zeros = x == 0.0f && y == 0.0f;
  float r = (x < y || isnan_(y)) ? x : y;
  return zeros ? (__builtin_signbit(x) ? x : y) : r;
}

// The rest of the C99 set with one exact answer (Section 1: the library
// covers all C99 real functions): sqrt correctly rounded (the IEEE square
// root; -0 -> -0, negative -> NaN), trunc, floor, ceil, round (halfway away
// from zero), rint (halfway to even), fabs, logb (the exponent of x as if
// normalized; 0 -> -inf, inf -> +inf), copysign, nextafter.
LMH_INLINE float sqrtf_f32(float x) { return __builtin_sqrtf(x); }
LMH_INLINE float truncf_f32(float x) { return trunc_(x); }
LMH_INLINE float floorf_f32(float x) { return __builtin_floorf(x); }
LMH_INLINE float ceilf_f32(float x) { return __builtin_ceilf(x); }
LMH_INLINE float rintf_f32(float x) { return rint_(x); }
LMH_INLINE float fabsf_f32(float x) { return fabs_(x); }
// round: x - trunc(x) is exact (both share x's exponent range), so the
// halfway test has no rounding; inf and NaN keep trunc's result
LMH_INLINE float roundf_f32(float x) {
  float t = trunc_(x);
  return fabs_(x - t) >= 0.5f ? t + copysign_(1.0f, x) : t;
}
LMH_INLINE float logbf_f32(float x) {
  float e = (float)(frexp_exp_(x) - 1);
  float r = isfinite_(x) ? e : fabs_(x);
  return x == 0.0f ? -__builtin_inff() : r;
}
LMH_INLINE float copysignf_f32(float x, float y) { return copysign_(x, y); }
// nextafter: the neighbour of x towards y by one step of the integer image
// (the magnitude grows when y lies beyond x away from zero); y when x == y,
// the smallest subnormal with y's sign from a zero, NaN if either is NaN
LMH_INLINE float nextafterf_f32(float x, float y) {
  bool away = (y > x) == (x > 0.0f);
  float r = as_f32(as_i32(x) + (away ? 1 : -1));
  r = x == 0.0f ? copysign_(0x1p-149f, y) : r;
  r = x == y ? y : r;
  return (isnan_(x) || isnan_(y)) ? x + y : r;
}

// C99 functions with integer operands or results (7.12.6): ldexp (=
// scalbn) x 2^n rounded once, n clamped to +-400 (beyond it every finite
// nonzero x already overflows or underflows); ilogb the exponent as if
// normalized, INT_MIN for 0 and NaN, INT_MAX for +-inf; frexp the mantissa
// in [0.5, 1) and exponent, (x, 0) for 0, inf and NaN
LMH_INLINE float ldexpf_f32(float x, int n) {
  return ldexp_(x, n < -400 ? -400 : (n > 400 ? 400 : n));
}
LMH_INLINE int ilogbf_f32(float x) {
  int e = frexp_exp_(x) - 1;
  e = isinf_(x) ? 2147483647 : e;
  return (x == 0 || isnan_(x)) ? (-2147483647 - 1) : e;
}
LMH_INLINE float frexp_mantf_f32(float x) { return frexp_mant_(x); }
LMH_INLINE int frexp_expf_f32(float x) { return isfinite_(x) ? frexp_exp_(x) : 0; }

// modf: the integral part trunc(x) and the fraction x - trunc(x) (exact),
// both with the sign of x; inf -> (+-0, +-inf), NaN -> (NaN, NaN).  fma: one
// IEEE fused multiply-add.  lrint / lround: rint(x) / round(x) as int64,
// INT64_MIN where it does not fit (and for NaN), as the x86-64 conversion.
LMH_INLINE float modf_fracf_f32(float x) {
  float f = x - trunc_(x);
  return copysign_(isinf_(x) ? 0.0f : f, x);
}
LMH_INLINE float modf_intf_f32(float x) { return trunc_(x); }
LMH_INLINE float fmaf_f32(float x, float y, float z) { return fma_(x, y, z); }
LMH_INLINE long long to_i64f_f32(float v) {
  bool fits = v >= -0x1p63f && v < 0x1p63f;               // false for NaN
  return fits ? (long long)v : (-9223372036854775807LL - 1);
}
LMH_INLINE long long lrintf_f32(float x) { return to_i64f_f32(rint_(x)); }
LMH_INLINE long long lroundf_f32(float x) { return to_i64f_f32(roundf_f32(x)); }

// remquo: the remainder is remainder(x, y); quo carries the sign of x / y
// and the low three bits of the quotient's magnitude rounded to nearest-even:
// r8 = |x| mod 8|y| exactly (|x| itself where 8|y| overflows), its quotient
// by |y| in [0, 7] from the exact signs of fma(-k, |y|, r8), then the same
// halfway rule as the remainder.  quo = 0 for the NaN cases and infinite y.
LMH_INLINE int remquo_quof_f32(float x, float y) {
  float n = fabs_(x), d = fabs_(y);
  float d8 = d * 8;                                   // exact or inf
  bool special = !isfinite_(x) || !isfinite_(d) || d == 0.0f;
  bool small = !(n >= d8);
  float r8 = fmodf_core(special || small ? 0.0f : n, special || small ? 1.0f : d8);
  r8 = small ? n : r8;
  int q = 0;
#pragma unroll
  for (int k = 1; k < 8; ++k) q += fma_(-(float)k, d, r8) >= 0.0f ? 1 : 0;
  float r = fma_(-(float)q, d, r8);                   // exact: r8 mod d
  float twice = r + r;
  q += (twice > d || (twice == d && (q & 1))) ? 1 : 0;
  q &= 7;
  q = (__builtin_signbit(x) != __builtin_signbit(y)) ? -q : q;
  return special ? 0 : q;
}

}  // namespace lmh

#pragma STDC FP_CONTRACT DEFAULT
