// Evaluators for data stored as bf16 or f16 (not in the paper, which covers
// binary64 and binary32): the input widened exactly to binary32, arithmetic
// in binary32 sized for the narrow formats, one rounding to the format at the
// end (by the storage type).  A bf16 or f16 result within 1.0 ULP needs the
// binary32 value within about 2^-12 relative (half an f16 ulp, with the
// final rounding's half ulp on top); every evaluator here stays below 2^-17,
// so the short polynomials and the binary32 transcendental unit (v_exp_f32,
// v_log_f32, v_rcp_f32, each within about one binary32 ulp) suffice where the
// binary32 evaluators spend double-length arithmetic.  Both formats have
// 65536 bit patterns; every one is checked against the oracle.
//
//   exp, exp2, log, log2, sinh, cosh, tanh: for bf16 and f16 (any binary32
//     value of those formats, bf16 subnormals included);
//   pow: for bf16 and f16, 2^(y log2|x|) with the binary32 Annex F selects;
//   sin, cos, tan, sincos: one Cody-Waite reduction by pi/2 below |x| =
//     65536 (every finite f16), the binary32 kernels' Payne-Hanek reduction
//     above (bf16 only), the same short polynomials after either;
//   atan2, atan, asin, acos: one reciprocal-unit quotient and a short atan
//     polynomial.
#pragma once
#include "eval_f32.h"
#include "generated/ph_table_bf16.inc"

#pragma STDC FP_CONTRACT OFF

namespace lmh {

// 2^t: v_exp_f32, with results below the binary32 normal range formed as
// 2^(t + 64) 2^-64 (one rounding into the subnormal range, 16 bits finer
// than bf16's)
LMH_INLINE float nexp2_core(float t) {
  bool lo = t < -125.0f;
  float y = exp2_hw(lo ? t + 64.0f : t);
  return lo ? ldexp_(y, -64) : y;
}

// e^x = 2^(x log2 e): the product's rounding moves the result by at most
// ln2 |t| 2^-24 relative (2^-17.2 at the bf16 underflow, t = -134)
LMH_INLINE float nexp(float x) { return nexp2_core(x * INVLN2_F_H); }

// 2^x; for an integer x the exact power of two, so that the results which
// are ties of the narrow formats' rounding (2^-25 in f16, 2^-134 in bf16)
// never hang on the last bit of v_exp_f32
LMH_INLINE float nexp2(float x) {
  float k = rint_(x);
  float c = k < -160.0f ? -160.0f : (k > 160.0f ? 160.0f : k);
  float y = nexp2_core(x);
  return x == k ? ldexp_(1.0f, (int)c) : y;
}

// log2 x from v_log_f32; binary32 subnormals (bf16 subnormals) of either
// sign are scaled by 2^64 first (v_log_f32 reads a subnormal as a zero of its
// sign, which would make log of a negative subnormal -inf instead of NaN).
// 0 -> -inf, negative -> NaN, inf -> inf.
LMH_INLINE float nlog2_core(float x) {
  bool sub = x != 0.0f && fabs_(x) < 0x1p-126f;
  float l = log2_hw(sub ? x * 0x1p64f : x);
  return sub ? l - 64.0f : l;
}

// log(1 + s) for |s| < 1/16 (s = x - 1 is exact there): Taylor to s^6, the
// omitted terms below s^6/7 < 2^-27 relative.  Near 1 the logarithm is small
// and an absolute error of v_log_f32 would be a large relative one.
LMH_INLINE float nlog1p_small(float s) {
  float p = fma_(s, fma_(s, fma_(s, fma_(s, -1.0f / 6.0f, 0.2f), -0.25f), 1.0f / 3.0f), -0.5f);
  return fma_(s * s, p, s);
}

LMH_INLINE float nlog(float x) {
  float s = x - 1.0f;
  float l = nlog2_core(x) * LN2_F_H;
  return fabs_(s) < 0.0625f ? nlog1p_small(s) : l;
}

LMH_INLINE float nlog2(float x) {
  float s = x - 1.0f;
  float l = nlog2_core(x);
  return fabs_(s) < 0.0625f ? nlog1p_small(s) * INVLN2_F_H : l;
}

// pow: t = y log2|x| with log2 within about 2^-21 relative (nlog2: the
// transcendental unit, or the series next to 1), so t is off by at most
// |t| 2^-20.9; a finite nonzero bf16 result has |t| < 134, an f16 one
// |t| < 25, so 2^t is within 2^-12.3 (bf16) and 2^-14.8 (f16) relative.
// Zeros, infinities, NaN, negative bases and the exact cases of Annex F come
// from the binary32 form's selects.
LMH_INLINE float npow(float x, float y) {
  float t = y * nlog2(fabs_(x));
  return powf_annexf(x, y, nexp2_core(t));
}

// e^a / 2 for a >= 0 (inf from a = 89.42 up)
LMH_INLINE float nexp_half(float a) { return exp2_hw(fma_(a, INVLN2_F_H, -1.0f)); }

// cosh x = e^|x|/2 + (1/4) / (e^|x|/2): a sum of positive terms
LMH_INLINE float ncosh(float x) {
  float e = nexp_half(fabs_(x));
  return e + 0.25f * rcp_hw(e);
}

// sinh: below |x| = 1/2 the Taylor series to x^5 (omitted terms below
// 2^-18.4 relative), above e^|x|/2 - (1/4) / (e^|x|/2), which cancels by at
// most a factor 1.6
LMH_INLINE float nsinh(float x) {
  float a = fabs_(x);
  float z = a * a;
  float p = fma_(a * z, fma_(z, 1.0f / 120.0f, 1.0f / 6.0f), a);
  float e = nexp_half(a);
  float big = e - 0.25f * rcp_hw(e);
  return copysign_(a < 0.5f ? p : big, x);
}

// tanh: below |x| = 0.55 the Taylor series to x^11 (omitted terms below
// 2^-18 relative); above 1 - 2 / (e^(2|x|) + 1), which does not cancel there
// (tanh 0.55 > 1/2) and reaches 1 once 2 / (e^(2|x|) + 1) is below half an ulp
LMH_INLINE float ntanh(float x) {
  float a = fabs_(x);
  float z = a * a;
  float p = fma_(z, fma_(z, fma_(z, fma_(z, -1382.0f / 155925.0f, 62.0f / 2835.0f),
                                  -17.0f / 315.0f), 2.0f / 15.0f), -1.0f / 3.0f);
  float small = fma_(a * z, p, a);
  float u = exp2_hw(a * (2.0f * INVLN2_F_H));
  float big = 1.0f - 2.0f * rcp_hw(u + 1.0f);
  return copysign_(a < 0.55f ? small : big, x);
}

// ---- f16 trigonometry ----------------------------------------------------
// k = rint(x 2/pi), r = x - k pi/2 by three chained FMAs on the binary32
// pieces of pi/2 (c0 the nearest float, c1 eight significant bits, c2 the
// nearest float to the rest), for |x| < 65536, which holds every finite f16
// and every bf16 the narrow kernels reduce this way.  Below 65536, |k| < 2^16
// and a nonzero k means |x| > pi/4, where both formats' values are multiples
// of 2^-11 or coarser: x - k c0 is then a multiple of 2^-23 below 1 in
// magnitude, so the first FMA is exact.  The second and third round once
// each, by at most 2^-24 of |r| + |k c2| (|k c2| < 2^-17), and the omitted
// k (pi/2 - c0 - c1 - c2) is below 2^-41: against the smallest reduced
// argument of these inputs, 2^-16 (x = 177.5), r is within 2^-23 relative.
// inf and NaN give a NaN r.
LMH_INLINE Trig32 hsincos_reduce(float x) {
  float k = rint_(x * TWO_OVER_PI_F);
  float r = fma_(k, -PIH_F_C2, fma_(k, -PIH_F_C1, fma_(k, -PIH_F_C0, x)));
  return Trig32{fff{r, 0.0f}, k};
}

// sin r and cos r for |r| <= pi/4 (a little more after k's rounding): Taylor
// to r^7 and to r^8 (omitted terms below 2^-20.9 and 2^-24 relative)
LMH_INLINE float hsin_poly(float r) {
  float z = r * r;
  return fma_(r * z, fma_(z, fma_(z, -1.0f / 5040.0f, 1.0f / 120.0f), -1.0f / 6.0f), r);
}
LMH_INLINE float hcos_poly(float r) {
  float z = r * r;
  return fma_(z, fma_(z, fma_(z, fma_(z, 1.0f / 40320.0f, -1.0f / 720.0f), 1.0f / 24.0f), -0.5f),
              1.0f);
}

// m = j mod 4 from q = j - 4 rint(j/4) in {-2, -1, 0, 1, 2} (exact: |j| is
// below 2^16); odd m takes the other polynomial, m in {2, 3} the sign
LMH_INLINE float hsin_finish(Trig32 s) {
  float r = s.r.hi;
  float q = s.j - 4.0f * rint_(s.j * 0.25f);
  bool odd = fabs_(q) == 1.0f;
  bool neg = fabs_(q) == 2.0f || q == -1.0f;
  float v = odd ? hcos_poly(r) : hsin_poly(r);
  return neg ? -v : v;
}

// tan: sin r / cos r (m even) or -cos r / sin r (m odd), each through the
// reciprocal unit (r = 0 only with m = 0)
LMH_INLINE float htan_finish(Trig32 s) {
  float r = s.r.hi;
  float q = s.j - 4.0f * rint_(s.j * 0.25f);
  bool odd = fabs_(q) == 1.0f;
  float sn = hsin_poly(r), cs = hcos_poly(r);
  return odd ? -cs * rcp_hw(sn) : sn * rcp_hw(cs);
}

// sin x = sin(r + m pi/2), cos x = sin(r + (m + 1) pi/2); sin(+-0) and
// tan(+-0) keep the sign of zero.  The state is either reduction's.
LMH_INLINE float nsin_fin(float x, Trig32 s) {
  float v = hsin_finish(s);
  return x == 0.0f ? x : v;
}
LMH_INLINE float ncos_fin(float, Trig32 s) {
  s.j += 1.0f;
  return hsin_finish(s);
}
LMH_INLINE float ntan_fin(float x, Trig32 s) {
  float v = htan_finish(s);
  return x == 0.0f ? x : v;
}

// ---- atan2, atan, asin, acos -----------------------------------------------
// t = min(|x|, |y|) / max(|x|, |y|) from the reciprocal unit on the larger
// one's mantissa (d = m 2^e: t = (n 2^-e) rcp(m), both factors in range
// whatever the exponents; a scaled numerator below the normal range rounds
// once at 2^-149, finer than either format), atan t = t + t^3 A(t^2) with A
// fitted to 2^-20.4 on [0, 1] (t within about 2^-22), then the binary32
// form's quadrant selects and Annex F cases.  atan x = atan2(x, 1); asin and
// acos from c = sqrt((1 - |x|)(1 + |x|)) by the square-root unit:
// asin x = atan2(x, c), acos x = atan2(c, x) (NaN beyond |x| = 1 through c).
LMH_INLINE float natan2(float y, float x) {
  float ay = fabs_(y), ax = fabs_(x);
  bool both_inf = isinf_(ax) && isinf_(ay);
  ay = both_inf ? 1.0f : ay;
  ax = both_inf ? 1.0f : ax;
  bool swap = ay > ax;
  float n = swap ? ax : ay, d = swap ? ay : ax;
  int e = frexp_exp_(d);
  float t = ldexp_(n, -e) * rcp_hw(frexp_mant_(d));
  float z = t * t;
  float a = fma_(t * z, poly_estrin(z, ATAN_N_F32), t);
  return atan2f_u35_finish(y, x, a, swap);
}

LMH_INLINE float natan(float x) { return natan2(x, 1.0f); }

LMH_INLINE float nasin_root(float x) {
  float a = fabs_(x);
  return __builtin_amdgcn_sqrtf((1.0f - a) * (1.0f + a));
}
LMH_INLINE float nasin(float x) { return natan2(x, nasin_root(x)); }
LMH_INLINE float nacos(float x) { return natan2(nasin_root(x), x); }

// f16: every finite argument is below 65536
LMH_INLINE float hsin(float x) { return nsin_fin(x, hsincos_reduce(x)); }
LMH_INLINE float hcos(float x) { return ncos_fin(x, hsincos_reduce(x)); }
LMH_INLINE float htan(float x) { return ntan_fin(x, hsincos_reduce(x)); }

// bf16 from 65536 up: Payne-Hanek in integer arithmetic.  |x| = m 2^(e-7)
// with m < 2^8 an integer (bf16 keeps 8 significant bits); the table word
// W(e) = floor(2^(e+55) 2/pi) mod 2^64 makes m W(e) mod 2^64 equal to
// 2|x|/pi in units of 2^-62, modulo 4: the quadrant in the top two bits, the
// fraction in the other 62, short of the exact value by less than m units
// (2^-54).  The fraction, taken to [-1/2, 1/2) with the quadrant rounded
// accordingly, is converted once to binary32 and multiplied by pi/2: r is
// within about 2^-22 relative of x - j pi/2 wherever the fraction exceeds
// 2^-30 (over all bf16 arguments it is at least 2^-13.3).  Negative x negates r
// and j; inf and NaN give a NaN r.  The state has the Cody-Waite path's
// meaning (r = x - j pi/2, j modulo 4).
LMH_INLINE Trig32 nbtrig_big(float x) {
  float a = fabs_(x);
  bool fin = isfinite_(a);
  int e = frexp_exp_(a) - 1;                          // a in [2^e, 2^(e+1))
  int row = e - PH_BF16_E0;
  row = row < 0 ? 0 : (row >= PH_BF16_ROWS ? PH_BF16_ROWS - 1 : row);
  unsigned m = (unsigned)(fin ? ldexp_(frexp_mant_(a), 8) : 128.0f);
  unsigned long long y = (unsigned long long)m * PH_WORDS_BF16[row];
  long long g = (long long)(y << 2) >> 2;             // the fraction, sign-extended
  float j = (float)(unsigned)(y >> 62) + (g < 0 ? 1.0f : 0.0f);
  float r = ((float)g * 0x1p-62f) * PIH_F_C0;
  r = fin ? r : __builtin_nanf("");
  return Trig32{fff{x < 0.0f ? -r : r, 0.0f}, x < 0.0f ? -j : j};
}

// bf16: from 65536 up (and for inf and NaN) the integer Payne-Hanek
// reduction above, below it the Cody-Waite reduction of f16
LMH_INLINE bool nbtrig_slow(float x) { return !(fabs_(x) < 65536.0f); }
LMH_INLINE Trig32 nbtrig_reduce(float x) {
  Trig32 s;
  if (nbtrig_slow(x))
    s = nbtrig_big(x);
  else
    s = hsincos_reduce(x);
  return s;
}

}  // namespace lmh

#pragma STDC FP_CONTRACT DEFAULT
