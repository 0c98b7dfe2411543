/* pow and atan2 for the oracle's fast C stages (fast32.c, fast64.c), in
 * double-double.  TEST INFRASTRUCTURE ONLY, like the rest of oracle/.
 *
 * Each core returns 1 with *rn set for the special cases (C99 Annex F:
 * NaN, infinities, zeros, and the values they fix), else 0 with the result
 * as the pair v times 2^k.
 *
 *  pow(x, z): the Annex F cases first, then |x|^z = e^w with w = z log|x|:
 *       log|x| = e ln 2 + 2 atanh((m - 1)/(m + 1)) for |x| = m 2^e,
 *       m in [1/sqrt 2, sqrt 2) (ln 2 in three doubles, the atanh series as
 *       in log), about 2^-100 relative; w = z log|x| as a pair; e^w =
 *       e^r 2^j with j = rint(w / ln 2) and r = w - j ln 2 (the Taylor
 *       series of e^r).  The error of w, at most |w| 2^-100 with |w| < 750
 *       where the result is neither 0 nor infinite, sets the bound: 2^-86
 *       relative.  The sign is negative for x < 0 and an odd integer z.
 *       Beyond the thresholds the caller passes (w above which the format
 *       overflows, below which it rounds to zero) the result is +-inf or
 *       +-0.
 *  atan2(y, x): the Annex F cases first; with a = |y|, b = |x| written
 *       m 2^e, t = min(a, b) / max(a, b) = (mantissa quotient, a pair)
 *       2^(difference of exponents); below 2^-62 atan t = t within 2^-124;
 *       otherwise three halvings atan t = 2 atan(t / (1 + sqrt(1 + t^2)))
 *       bring t under tan(pi/32) and the series t sum (-t^2)^k/(2k+1),
 *       k <= 18, ends it (first omitted term below 2^-127 of the sum);
 *       then pi/2 - atan for a > b, pi - atan for x < 0 and the sign of y,
 *       all in pairs (pi/2 from three doubles): about 2^-98 relative,
 *       bound 2^-90. */
#pragma once
#include "common.h"

static int is_int_d(double z) { return isfinite(z) && nearbyint(z) == z; }
static int is_odd_d(double z) { return is_int_d(z) && fabs(z) < 0x1p53 && fmod(z, 2.0) != 0.0; }

/* sqrt of a pair a >= 1: one Newton step on the binary64 square root */
static dd dd_sqrt(dd a) {
  double r0 = sqrt(a.hi);
  dd q = dd_add(a, dd_neg(two_prod(r0, r0)));
  return dd_add(dd_from(r0), dd_from(q.hi / (2.0 * r0)));
}

/* log a for a finite a > 0, a != 1, as a pair */
static dd log_pair(double a) {
  int e;
  double m = frexp(a, &e);
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  dd t = dd_div(dd_from(m - 1.0), two_sum(m, 1.0));
  dd l = atanh2_series(t);
  dd el = dd_add(two_prod((double)e, LN2_D[0]), two_prod((double)e, LN2_D[1]));
  el = dd_add(el, dd_from((double)e * LN2_D[2]));
  return dd_add(el, l);
}

/* e^w for a pair |w| < 750 as v 2^k: j = rint(w / ln 2), r = w - j ln 2 (ln 2
   in three doubles), the Taylor series of e^r */
static void exp_of_pair(dd w, dd* v, int* k) {
  double j = nearbyint(w.hi / LN2_D[0]);
  dd r = dd_add(w, dd_neg(two_prod(j, LN2_D[0])));
  r = dd_add(r, dd_neg(two_prod(j, LN2_D[1])));
  r = dd_add(r, dd_from(-j * LN2_D[2]));
  *v = exp_series(r);
  *k = (int)j;
}

static int pow_core(double x, double z, double w_over, double w_zero, dd* v, int* k, double* rn) {
  *k = 0;
  if (z == 0.0 || x == 1.0) {
    *rn = 1.0;
    return 1;
  }
  if (isnan(x) || isnan(z)) {
    *rn = NAN;
    return 1;
  }
  double ax = fabs(x);
  int odd = is_odd_d(z);
  if (isinf(z)) {
    *rn = ax == 1.0 ? 1.0 : ((ax < 1.0) == (z < 0.0) ? INFINITY : 0.0);
    return 1;
  }
  if (x == 0.0) {
    *rn = z < 0.0 ? (odd ? copysign(INFINITY, x) : INFINITY) : (odd ? x : 0.0);
    return 1;
  }
  if (isinf(x)) {
    double mag = z < 0.0 ? 0.0 : INFINITY;
    *rn = (x < 0.0 && odd) ? -mag : mag;
    return 1;
  }
  if (x < 0.0 && !is_int_d(z)) {
    *rn = NAN;
    return 1;
  }
  double sgn = (x < 0.0 && odd) ? -1.0 : 1.0;
  dd l = log_pair(ax);
  if (!(fabs(l.hi * z) < 1e5)) { /* far beyond either threshold (the pair product would overflow) */
    *rn = sgn * (l.hi * z > 0.0 ? INFINITY : 0.0);
    return 1;
  }
  dd w = dd_mul_d(l, z);
  if (w.hi > w_over) {
    *rn = sgn * INFINITY;
    return 1;
  }
  if (w.hi < w_zero) {
    *rn = sgn * 0.0;
    return 1;
  }
  dd s;
  exp_of_pair(w, &s, k);
  *v = sgn < 0.0 ? dd_neg(s) : s;
  return 0;
}

/* atan t for a pair 2^-62 <= t <= 1 */
static dd atan_pair(dd t) {
  for (int i = 0; i < 3; ++i) {
    dd s = dd_sqrt(dd_add(dd_from(1.0), dd_mul(t, t)));
    t = dd_div(t, dd_add(dd_from(1.0), s));
  }
  dd z = dd_neg(dd_mul(t, t));
  dd a = dd_mul(horner(z, INV_ODD, 1, 0, 18, 9), t);
  a.hi *= 8.0;
  a.lo *= 8.0;
  return a;
}

static int atan2_core(double y, double x, dd* v, int* k, double* rn) {
  *k = 0;
  dd pio2 = {PIO2_D[0], PIO2_D[1]};
  dd pi = {2.0 * PIO2_D[0], 2.0 * PIO2_D[1]};
  dd pio4 = {0.5 * PIO2_D[0], 0.5 * PIO2_D[1]};
  if (isnan(x) || isnan(y)) {
    *rn = NAN;
    return 1;
  }
  int special = 0;
  dd s = {0.0, 0.0};
  if (y == 0.0) {
    if (x > 0.0 || (x == 0.0 && !signbit(x))) {
      *rn = y;
      return 1;
    }
    s = pi;
    special = 1;
  } else if (isinf(y)) {
    s = isinf(x) ? (x > 0.0 ? pio4 : dd_add(pio2, pio4)) : pio2;
    special = 1;
  } else if (x == 0.0) {
    s = pio2;
    special = 1;
  } else if (isinf(x)) {
    if (x > 0.0) {
      *rn = copysign(0.0, y);
      return 1;
    }
    s = pi;
    special = 1;
  }
  if (special) {
    *v = signbit(y) ? dd_neg(s) : s;
    return 0;
  }
  double a = fabs(y), b = fabs(x);
  int swap = a > b;
  double n = swap ? b : a, d = swap ? a : b;
  int en, ed;
  double mn = frexp(n, &en), md = frexp(d, &ed);
  dd q = dd_div(dd_from(mn), dd_from(md));
  int sh = en - ed;
  if (sh < -62 && !swap && x > 0.0) { /* atan t = t within 2^-124 */
    *v = y < 0.0 ? dd_neg(q) : q;
    *k = sh;
    return 0;
  }
  dd t = {ldexp(q.hi, sh), ldexp(q.lo, sh)};
  dd r = sh < -62 ? t : atan_pair(t);
  if (swap) r = dd_add(pio2, dd_neg(r));
  if (x < 0.0) r = dd_add(pi, dd_neg(r));
  *v = y < 0.0 ? dd_neg(r) : r;
  return 0;
}

/* asin, acos and atan for the fast stages: atan x = atan2(x, 1); asin and
 * acos through s = sqrt((1 - |x|)(1 + |x|)) as a pair and the atan of the
 * smaller-to-larger quotient of (|x|, s), as in atan2 (asin x = atan2(x, s),
 * acos x = atan2(s, x)); below |x| = 2^-30, asin x = x + x^3/6 and acos x =
 * pi/2 - x - x^3/6 (the next terms are under 2^-120 relative).  Bound
 * 2^-90 relative, the same as atan2's. */

/* atan2 of two pairs a, b >= 0 with max(a, b) > 0 */
static dd atan2_pos(dd a, dd b) {
  dd pio2 = {PIO2_D[0], PIO2_D[1]};
  int swap = a.hi > b.hi;
  dd n = swap ? b : a, d = swap ? a : b;
  dd t = dd_div(n, d);
  dd r = t.hi < 0x1p-62 ? t : atan_pair(t);
  return swap ? dd_add(pio2, dd_neg(r)) : r;
}

/* sqrt((1 - a)(1 + a)) for 0 <= a < 1, as a pair */
static dd cos_of_asin(double a) {
  dd p = dd_mul(two_sum(1.0, -a), two_sum(1.0, a));
  return dd_sqrt(p);
}

static int asin_core(double x, dd* v, int* k, double* rn) {
  *k = 0;
  double a = fabs(x);
  if (isnan(x) || a > 1.0) {
    *rn = NAN;
    return 1;
  }
  if (x == 0.0) {
    *rn = x;
    return 1;
  }
  dd r;
  if (a == 1.0) {
    r = (dd){PIO2_D[0], PIO2_D[1]};
  } else if (a < 0x1p-30) {
    r = fast_two_sum(a, a * a * a / 6.0);
  } else {
    r = atan2_pos(dd_from(a), cos_of_asin(a));
  }
  *v = x < 0.0 ? dd_neg(r) : r;
  return 0;
}

static int acos_core(double x, dd* v, int* k, double* rn) {
  *k = 0;
  double a = fabs(x);
  dd pio2 = {PIO2_D[0], PIO2_D[1]};
  dd pi = {2.0 * PIO2_D[0], 2.0 * PIO2_D[1]};
  if (isnan(x) || a > 1.0) {
    *rn = NAN;
    return 1;
  }
  if (x == 1.0) {
    *rn = 0.0;
    return 1;
  }
  if (x == -1.0) {
    *v = pi;
    return 0;
  }
  if (a < 0x1p-30) {
    *v = dd_add(pio2, dd_neg(fast_two_sum(x, x * x * x / 6.0)));
    return 0;
  }
  dd r = atan2_pos(cos_of_asin(a), dd_from(a));
  *v = x < 0.0 ? dd_add(pi, dd_neg(r)) : r;
  return 0;
}

static int atan_core(double x, dd* v, int* k, double* rn) { return atan2_core(x, 1.0, v, k, rn); }


/* log10, log1p, exp10, expm1 and cbrt for the fast stages (bound 2^-90):
 *  log10 x = log x / ln 10 (1/ln 10 as a pair from log_pair(10));
 *  log1p x = x - x^2/2 + x^3/3 below |x| = 2^-40, 2 atanh(x / (2 + x))
 *       for -0.29 < x < 0.41 (the quotient as a pair, within 0.171), else
 *       log(1 + x) with 1 + x an exact pair (log of a pair: log of its head
 *       plus lo/hi);
 *  exp10 x = e^(x ln 10) (ln 10 as a pair), as pow's exponential;
 *  expm1 x = x sum x^n/(n+1)! for |x| < 0.3 (22 terms), else e^x - 1 with
 *       the 1 subtracted from the scaled pair;
 *  cbrt x: |x| = a 2^(3q) with a in [0.5, 4), one Newton step in pairs from
 *       the host's cbrt of a (error squared: about 2^-103), times 2^q.
 * Beyond the caller's thresholds (w above which the format overflows, below
 * which e^w rounds to zero) exp10 and expm1 give inf, 0 or -1. */
static dd LN10_P, INV_LN10_P;

__attribute__((constructor)) static void init_ln10(void) {
  LN10_P = log_pair(10.0);
  INV_LN10_P = dd_div(dd_from(1.0), LN10_P);
}

static dd log_of_pair(dd a) {
  dd l = a.hi == 1.0 ? dd_from(0.0) : log_pair(a.hi);
  return dd_add(l, dd_from(a.lo / a.hi));
}

static int log_specials(double x, double* rn) {
  if (isnan(x)) {
    *rn = x;
    return 1;
  }
  if (x < 0.0) {
    *rn = NAN;
    return 1;
  }
  if (x == 0.0) {
    *rn = -INFINITY;
    return 1;
  }
  if (isinf(x)) {
    *rn = x;
    return 1;
  }
  return 0;
}

static int log10_core(double x, dd* v, int* k, double* rn) {
  *k = 0;
  if (log_specials(x, rn)) return 1;
  if (x == 1.0) {
    *rn = 0.0;
    return 1;
  }
  *v = dd_mul(log_pair(x), INV_LN10_P);
  return 0;
}

static int log1p_core(double x, dd* v, int* k, double* rn) {
  *k = 0;
  if (isnan(x) || x < -1.0) {
    *rn = NAN;
    return 1;
  }
  if (x == -1.0) {
    *rn = -INFINITY;
    return 1;
  }
  if (x == 0.0 || isinf(x)) {
    *rn = x;
    return 1;
  }
  if (fabs(x) < 0x1p-40) {
    double t = x * x;
    *v = fast_two_sum(x, t * (x / 3.0 - 0.5));
    return 0;
  }
  if (x > -0.29 && x < 0.41) { /* 2 atanh(x / (2 + x)), the quotient within 0.171 */
    *v = atanh2_series(dd_div(dd_from(x), two_sum(2.0, x)));
    return 0;
  }
  *v = log_of_pair(two_sum(1.0, x));
  return 0;
}

static int exp10_core(double x, double w_over, double w_zero, dd* v, int* k, double* rn) {
  *k = 0;
  if (isnan(x)) {
    *rn = x;
    return 1;
  }
  if (x == 0.0 || !(fabs(x) < 400.0)) { /* beyond 400 it overflows or rounds to 0 */
    *rn = x == 0.0 ? 1.0 : (x > 0.0 ? INFINITY : 0.0);
    return 1;
  }
  dd w = dd_mul_d(LN10_P, x);
  if (w.hi > w_over) {
    *rn = INFINITY;
    return 1;
  }
  if (w.hi < w_zero) {
    *rn = 0.0;
    return 1;
  }
  exp_of_pair(w, v, k);
  return 0;
}

static int expm1_core(double x, double w_over, dd* v, int* k, double* rn) {
  *k = 0;
  if (isnan(x) || x == 0.0) {
    *rn = x;
    return 1;
  }
  if (x > w_over) {
    *rn = INFINITY;
    return 1;
  }
  if (x < -800.0) {
    *rn = -1.0;
    return 1;
  }
  if (fabs(x) < 0.3) {
    *v = dd_mul_d(horner(dd_from(x), INV_FACT, 1, 1, 21, 13), x);
    return 0;
  }
  dd e;
  int j;
  exp_of_pair(dd_from(x), &e, &j);
  if (x > 0.0) {
    *v = dd_add(e, dd_from(-ldexp(1.0, -j)));
    *k = j;
  } else {
    *v = dd_add(dd_from(-1.0), (dd){ldexp(e.hi, j), ldexp(e.lo, j)});
  }
  return 0;
}

static int cbrt_core(double x, dd* v, int* k, double* rn) {
  *k = 0;
  if (isnan(x) || x == 0.0 || isinf(x)) {
    *rn = x;
    return 1;
  }
  int e;
  double m = frexp(fabs(x), &e);
  int q = (e + 3000) / 3 - 1000; /* floor(e / 3) */
  double a = ldexp(m, e - 3 * q); /* [0.5, 4) */
  double y0 = cbrt(a);
  dd y2 = two_prod(y0, y0);
  dd t = dd_add(dd_mul_d(y2, y0), dd_from(-a));
  dd y = fast_two_sum(y0, -t.hi / (3.0 * y2.hi));
  *v = x < 0.0 ? dd_neg(y) : y;
  *k = q;
  return 0;
}

/* asinh, acosh and atanh for the fast stages (bound 2^-90), through
 * log1p of a pair w in (-0.29, 0.41) as 2 atanh(w / (2 + w)) and log of a
 * pair elsewhere:
 *  asinh a (a = |x|) = x - x^3/6 below 2^-30, log1p(a + a^2/(1 + sqrt(1 +
 *       a^2))) below 0.4, log(a + sqrt(a^2 + 1)) to 2^500, log 2a beyond;
 *  acosh x = log1p((x - 1) + sqrt((x - 1)(x + 1))) while that argument is
 *       below 0.41, log(x + sqrt(x^2 - 1)) to 2^500, log 2x beyond;
 *  atanh x = (2 atanh x)/2 by the series to |x| = 0.171, else
 *       log((1 + x)/(1 - x)) / 2 with the quotient as a pair. */
static dd log1p_pair(dd w) { return atanh2_series(dd_div(w, dd_add(dd_from(2.0), w))); }

static int asinh_core(double x, dd* v, int* k, double* rn) {
  *k = 0;
  if (isnan(x) || isinf(x) || x == 0.0) {
    *rn = x;
    return 1;
  }
  double a = fabs(x);
  dd r;
  if (a < 0x1p-30) {
    r = fast_two_sum(a, -(a * a * a) / 6.0);
  } else if (a > 0x1p500) {
    r = dd_add(log_pair(a), (dd){LN2_D[0], LN2_D[1]});
  } else {
    dd a2 = two_prod(a, a);
    dd s = dd_sqrt(dd_add(a2, dd_from(1.0)));
    if (a < 0.4) {
      dd w = dd_add(dd_from(a), dd_div(a2, dd_add(dd_from(1.0), s)));
      r = log1p_pair(w);
    } else {
      r = log_of_pair(dd_add(dd_from(a), s));
    }
  }
  *v = x < 0.0 ? dd_neg(r) : r;
  return 0;
}

static int acosh_core(double x, dd* v, int* k, double* rn) {
  *k = 0;
  if (isnan(x) || x < 1.0) {
    *rn = NAN;
    return 1;
  }
  if (x == 1.0 || isinf(x)) {
    *rn = x == 1.0 ? 0.0 : x;
    return 1;
  }
  if (x > 0x1p500) {
    *v = dd_add(log_pair(x), (dd){LN2_D[0], LN2_D[1]});
    return 0;
  }
  dd xm = two_sum(x, -1.0);
  dd s = dd_sqrt(dd_mul(xm, two_sum(x, 1.0)));
  dd w = dd_add(xm, s);
  *v = w.hi < 0.41 ? log1p_pair(w) : log_of_pair(dd_add(dd_from(x), s));
  return 0;
}

static int atanh_core(double x, dd* v, int* k, double* rn) {
  *k = 0;
  double a = fabs(x);
  if (isnan(x) || a > 1.0) {
    *rn = NAN;
    return 1;
  }
  if (x == 0.0 || a == 1.0) {
    *rn = x == 0.0 ? x : copysign(INFINITY, x);
    return 1;
  }
  dd r;
  if (a <= 0.171) {
    r = atanh2_series(dd_from(x));
  } else {
    r = log_of_pair(dd_div(two_sum(1.0, x), two_sum(1.0, -x)));
  }
  r.hi *= 0.5;
  r.lo *= 0.5;
  *v = r;
  return 0;
}

/* erf and erfc for the fast stages (bound 2^-90):
 *  below |x| = 2^-30, erf x = (2/sqrt pi) x (1 - x^2/3);
 *  below 2, erf a = (2/sqrt pi) e^(-a^2) sum_n (2a^2)^n a / (1 3 ... (2n+1))
 *       (positive terms, summed until the next is below 2^-110 of the sum);
 *  from 2 to 30, erfc a = e^(-a^2)/sqrt(pi) / (a + (1/2)/(a + 1/(a + (3/2)/
 *       (a + ...)))), the continued fraction evaluated from depth 200 (its
 *       truncation error is below 2^-107 from a = 2 on), as v 2^k;
 *  erf = 1 - erfc and erfc = 1 - erf (or 2 - erfc(|x|) for negative x)
 *  where the other one is the one computed; beyond |x| = 27 erf is +-1 and
 *  erfc(x) 2 within 2^-1000, and erfc(x) for x >= 30 rounds to 0. */
static dd INV_SQRTPI_P;

__attribute__((constructor)) static void init_sqrtpi(void) {
  dd pi = {2.0 * PIO2_D[0], 2.0 * PIO2_D[1]};
  INV_SQRTPI_P = dd_div(dd_from(1.0), dd_sqrt(pi));
}

static void erfc_cf(double a, dd* v, int* k) {
  dd t = dd_from(a);
  for (int n = 200; n >= 1; --n) t = dd_add(dd_from(a), dd_div(dd_from(0.5 * n), t));
  dd e;
  exp_of_pair(dd_neg(two_prod(a, a)), &e, k);
  *v = dd_div(dd_mul(e, INV_SQRTPI_P), t);
}

static dd erf_small(double a) { /* 0 < a < 2 */
  dd tw = {2.0 * INV_SQRTPI_P.hi, 2.0 * INV_SQRTPI_P.lo};
  if (a < 0x1p-30) return dd_add(dd_mul_d(tw, a), dd_from(-tw.hi * a * a * a / 3.0));
  dd q = two_prod(2.0 * a, a);
  dd term = dd_from(a), sum = dd_from(a);
  for (int n = 0; n < 400; ++n) {
    term = dd_div(dd_mul(term, q), dd_from(2.0 * n + 3.0));
    sum = dd_add(sum, term);
    if (term.hi < 0x1p-110 * sum.hi) break;
  }
  dd e;
  int k;
  exp_of_pair(dd_neg(two_prod(a, a)), &e, &k);
  e.hi = ldexp(e.hi, k);
  e.lo = ldexp(e.lo, k);
  return dd_mul(dd_mul(sum, e), tw);
}

static int erf_core(double x, dd* v, int* k, double* rn) {
  *k = 0;
  double a = fabs(x);
  if (isnan(x) || x == 0.0) {
    *rn = x;
    return 1;
  }
  if (a > 27.0) { /* erfc below 2^-1000 */
    *rn = copysign(1.0, x);
    return 1;
  }
  dd r;
  if (a < 0x1p-900) { /* (2/sqrt pi) a, formed at a 2^600 so that no part is subnormal */
    dd tw = {2.0 * INV_SQRTPI_P.hi, 2.0 * INV_SQRTPI_P.lo};
    r = dd_mul_d(tw, a * 0x1p600);
    *k = -600;
  } else if (a < 2.0) {
    r = erf_small(a);
  } else {
    dd c;
    int j;
    erfc_cf(a, &c, &j);
    r = dd_add(dd_from(1.0), dd_neg((dd){ldexp(c.hi, j), ldexp(c.lo, j)}));
  }
  *v = x < 0.0 ? dd_neg(r) : r;
  return 0;
}

static int erfc_core(double x, dd* v, int* k, double* rn) {
  *k = 0;
  double a = fabs(x);
  if (isnan(x)) {
    *rn = x;
    return 1;
  }
  if (x == 0.0 || x <= -27.0 || x >= 30.0) {
    *rn = x == 0.0 ? 1.0 : (x < 0.0 ? 2.0 : 0.0);
    return 1;
  }
  if (a < 2.0) {
    dd e = erf_small(a);
    *v = dd_add(dd_from(1.0), x < 0.0 ? e : dd_neg(e));
    return 0;
  }
  dd c;
  int j;
  erfc_cf(a, &c, &j);
  if (x > 0.0) {
    *v = c;
    *k = j;
  } else {
    *v = dd_add(dd_from(2.0), dd_neg((dd){ldexp(c.hi, j), ldexp(c.lo, j)}));
  }
  return 0;
}

/* ---- lgamma and tgamma ------------------------------------------------------
 * C99's lgamma and tgamma (the paper's library covers the C99 real
 * functions, Section 1, and does not describe these two).  Textbook
 * definitions, in pairs:
 *
 *  log Gamma(z), z > 0: z + n = y with y >= 20 and n >= 0 the smallest such
 *       integer; log Gamma(z) = log Gamma(y) - log(z (z + 1) ... (z + n - 1))
 *       (Gamma(t + 1) = t Gamma(t)), and Stirling's series
 *       log Gamma(y) = (y - 1/2) log y - y + log(2 pi)/2
 *                      + sum_{k=1..15} B_2k / (2k (2k - 1) y^(2k - 1)),
 *       whose first omitted term is below 2^-110 at y = 20 (B_2k the
 *       Bernoulli numbers, exact rationals).
 *  z < 0, not an integer: Gamma(z) Gamma(1 - z) = pi / sin(pi z), so
 *       log|Gamma(z)| = log pi - log|sin(pi z)| - log Gamma(1 - z), with
 *       |sin(pi z)| = sin(pi |f|) for the exact fraction f = z - rint(z)
 *       (cos(pi (1/2 - |f|)) above |f| = 1/4, so the series run on at most
 *       pi/4).
 *  Gamma(z) = sign e^(log|Gamma(z)|), the sign negative on the intervals
 *       (-2m - 1, -2m).
 * The pieces carry relative errors of at most about 2^-98 each; the bound
 * kept per element is absolute, 2^-96 times the sum of the magnitudes of
 * the terms added, so that near the zeros of log Gamma (z = 1, 2 and two
 * on each negative interval from (-3, -2) on) the relative bound of the
 * result grows as the result shrinks and the rounding test sees it.
 * Exact cases: log Gamma(1) = log Gamma(2) = +0; the poles and the C99
 * special values (lgamma(+-0) = lgamma(-n) = lgamma(+-inf) = +inf,
 * tgamma(+-0) = +-inf, tgamma(-n) = tgamma(-inf) = NaN, tgamma(+inf) =
 * +inf). */
static const double BERN_NUM[15] = {1.0, -1.0, 1.0, -1.0, 5.0, -691.0, 7.0, -3617.0, 43867.0,
                                    -174611.0, 854513.0, -236364091.0, 8553103.0,
                                    -23749461029.0, 8615841276005.0};
static const double BERN_DEN[15] = {6.0, 30.0, 42.0, 30.0, 66.0, 2730.0, 6.0, 510.0, 798.0,
                                    330.0, 138.0, 2730.0, 6.0, 870.0, 14322.0};
static dd STIRLING_C[15], HALF_LN_2PI, LN_PI, PI_PAIR;

__attribute__((constructor)) static void init_gamma(void) {
  for (int k = 1; k <= 15; ++k)
    STIRLING_C[k - 1] = dd_div(dd_from(BERN_NUM[k - 1]),
                               dd_from(BERN_DEN[k - 1] * (2.0 * k) * (2.0 * k - 1.0)));
  PI_PAIR = (dd){2.0 * PIO2_D[0], 2.0 * PIO2_D[1]};
  LN_PI = log_of_pair(PI_PAIR);
  HALF_LN_2PI = log_of_pair((dd){2.0 * PI_PAIR.hi, 2.0 * PI_PAIR.lo});
  HALF_LN_2PI.hi *= 0.5;
  HALF_LN_2PI.lo *= 0.5;
}

/* log Gamma(z) for a pair z > 0 (finite), with *err its absolute error bound */
static dd lgamma_pos(dd z, double* err) {
  dd y = z, p = dd_from(1.0);
  int n = 0;
  while (y.hi < 20.0) {
    p = n ? dd_mul(p, y) : y;
    y = dd_add(y, dd_from(1.0));
    ++n;
  }
  dd ly = log_of_pair(y);
  dd a = dd_mul(dd_add(y, dd_from(-0.5)), ly);
  dd u = dd_div(dd_from(1.0), y);
  dd u2 = dd_mul(u, u);
  dd s = STIRLING_C[14];
  for (int k = 13; k >= 0; --k) s = dd_add(dd_mul(s, u2), STIRLING_C[k]);
  s = dd_mul(s, u);
  dd l = dd_add(dd_add(a, dd_neg(y)), dd_add(HALF_LN_2PI, s));
  double e = fabs(a.hi) + fabs(y.hi) + 1.0;
  if (n) {
    dd lp = log_of_pair(p);
    l = dd_add(l, dd_neg(lp));
    e += fabs(lp.hi) + 1.0;
  }
  *err = 0x1p-96 * e;
  return l;
}

/* log|Gamma(x)| for a finite x that is not 0 or a negative integer, as the
   pair times 2^k (k = 16 above x = 2^1000, where the value nears or passes
   the binary64 range; else 0), with *err the absolute error bound of the
   pair.  Below |x| = 2^-500 (binary64 arguments only) log Gamma(x) =
   log Gamma(1 + x) - log x and log|sin(pi x)| = log pi + log|x| (the
   relative error of sin(pi x) ~ pi x there is below 2^-996), so that no
   product runs through the subnormal range. */
static dd lgamma_any(double x, double* err, int* k) {
  *k = 0;
  if (x > 0x1p1000) { /* Stirling's series alone; its sum is below 2^-1003 */
    dd ly = log_pair(x);
    dd ym = dd_add(dd_from(x), dd_from(-0.5));
    ym.hi = ldexp(ym.hi, -16);
    ym.lo = ldexp(ym.lo, -16);
    dd a = dd_mul(ym, ly);
    double ys = ldexp(x, -16);
    dd c = {ldexp(HALF_LN_2PI.hi, -16), ldexp(HALF_LN_2PI.lo, -16)};
    *k = 16;
    *err = 0x1p-96 * (fabs(a.hi) + ys + 1.0);
    return dd_add(dd_add(a, dd_from(-ys)), c);
  }
  if (x > 0.0 && x < 0x1p-500) {
    double e1;
    dd lg = lgamma_pos(two_sum(x, 1.0), &e1);
    dd lx = log_pair(x);
    *err = e1 + 0x1p-96 * (fabs(lx.hi) + 1.0);
    return dd_add(lg, dd_neg(lx));
  }
  if (x > 0.0) return lgamma_pos(dd_from(x), err);
  double f = fabs(x - nearbyint(x));
  dd ls;
  if (f < 0x1p-500)
    ls = dd_add(LN_PI, log_pair(f));
  else
    ls = log_of_pair(f <= 0.25 ? sin_series(dd_mul_d(PI_PAIR, f))
                               : cos_series(dd_mul_d(PI_PAIR, 0.5 - f)));
  double e1;
  dd lg = lgamma_pos(two_sum(1.0, -x), &e1);
  *err = e1 + 0x1p-96 * (fabs(LN_PI.hi) + fabs(ls.hi) + 1.0);
  return dd_add(dd_add(LN_PI, dd_neg(ls)), dd_neg(lg));
}

static int is_pole(double x) { return x == 0.0 || (x < 0.0 && nearbyint(x) == x); }

/* lgamma: 1 with *rn for the exact cases, else 0 with the value v 2^k and
   *rel, the relative error bound of v */
static int lgamma_core(double x, dd* v, int* k, double* rel, double* rn) {
  if (isnan(x)) {
    *rn = x;
    return 1;
  }
  if (isinf(x) || is_pole(x)) {
    *rn = INFINITY;
    return 1;
  }
  if (x == 1.0 || x == 2.0) {
    *rn = 0.0;
    return 1;
  }
  double err;
  *v = lgamma_any(x, &err, k);
  *rel = err / fabs(v->hi);
  return 0;
}

/* tgamma: 1 with *rn for the exact cases and for log|Gamma| above w_over
   (the format overflows) or below w_zero (the result rounds to zero), else
   0 with the value v 2^k and *rel */
static int tgamma_core(double x, double w_over, double w_zero, dd* v, int* k, double* rel,
                       double* rn) {
  if (isnan(x)) {
    *rn = x;
    return 1;
  }
  if (x == 0.0) {
    *rn = copysign(INFINITY, x);
    return 1;
  }
  if (x == -INFINITY || is_pole(x)) {
    *rn = NAN;
    return 1;
  }
  if (x == INFINITY) {
    *rn = INFINITY;
    return 1;
  }
  double sgn = (x < 0.0 && fmod(floor(x), 2.0) != 0.0) ? -1.0 : 1.0;
  double err;
  int kw;
  dd w = lgamma_any(x, &err, &kw);
  if (kw || w.hi > w_over || w.hi < w_zero) { /* kw != 0: x > 2^1000 */
    *rn = sgn * (kw || w.hi > w_over ? INFINITY : 0.0);
    return 1;
  }
  exp_of_pair(w, v, k);
  if (sgn < 0.0) *v = dd_neg(*v);
  *rel = 1.01 * err + 0x1p-98;
  return 0;
}
