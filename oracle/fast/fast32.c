/* Fast first stage of the oracle for binary32 sin, cos, tan, exp, exp2, log,
 * log2, sinh, cosh and tanh.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/ to sweep every binary32 input;
 * the GPU library never links or calls it, and it shares no code, header,
 * table or constant generator with the library (its constants come from
 * oracle.consts through oracle/fast/make_tables.py).
 *
 * Each function returns the exact value as a double-double v = hi + lo with
 * |v - f(x)| <= 2^-90 |f(x)| (the claimed bound, checked in
 * tests/test_oracle_fast.py against the ball oracle), and the correctly
 * rounded binary32 result when that bound decides it; otherwise it reports
 * the input as undecided and the caller asks the ball oracle.
 *
 *  sin: 2|x|/pi = k + f (|f| <= 1/2) from an integer product of the 24-bit
 *       mantissa with 256 bits of 2/pi (the Payne-Hanek idea of the paper's
 *       Section 5 done in exact integer arithmetic), r = f pi/2 in
 *       double-double, then the Taylor series of sin r or cos r
 *       (|r| <= pi/4) by quadrant.
 *  exp: x = k ln2 + r, |r| <= ln2/2, ln 2 as three doubles (k ln2_0 exact),
 *       e^r by its Taylor series in double-double, times 2^k.
 *  log: x = m 2^e, m in [1/sqrt 2, sqrt 2); log m = 2 atanh t,
 *       t = (m - 1)/(m + 1), by its series in double-double, plus e ln 2.
 *  cos, tan: sin's reduction; cos |x| = sin(|x| + pi/2), tan = sin r / cos r
 *       or -cos r / sin r by the quadrant's parity.
 *  exp2: 2^(k + f) = 2^k e^(f ln 2); log2 = log / ln 2 (powers of two exact).
 *  sinh, cosh, tanh: from e^|x| and its reciprocal as pairs; below 2^-4
 *       sinh by its Taylor series and tanh = sinh / sqrt(1 + sinh^2).
 *
 * Error budget (relative): the double-double operations of a series of
 * n <= 40 terms contribute below n 2^-104; the reductions are exact or below
 * 2^-97 (sin: the 128 fraction bits kept, 2^-128 absolute, against the
 * smallest reduced argument of a binary32 input, about 2^-31); the constants
 * are within 2^-150.  2^-90 leaves a factor of 2^5 to spare.
 *
 * Built with -ffp-contract=off so that the error-free transformations stay
 * exact (the exact product's error term by C99 fma(), which -mfma makes the
 * host's fused multiply-add instruction).
 */
#define _GNU_SOURCE /* exp10 in the host libm */
#include "binary.h"

/* |x| = m 2^E (m < 2^24 an integer): 2|x|/pi = q + f with q an integer taken
   modulo 4 and |f| <= 1/2, f as a pair (absolute error below 2^-127) */
static dd reduce_2_over_pi(uint32_t m, int E, int* quadrant) {
  /* bits of 2/pi of weight 2^-i with i <= E - 2 contribute multiples of 4:
     start the 256-bit window W at weight 2^-s */
  int s = E - 1 > 1 ? E - 1 : 1;
  uint32_t w[8];
  for (int i = 0; i < 8; ++i) w[i] = tbits32(s - 1 + 32 * i);
  /* P = m W (288 bits) as little-endian 64-bit words; value = P 2^(E - s - 255) */
  uint64_t Q[5] = {0, 0, 0, 0, 0};
  uint64_t carry = 0;
  for (int i = 7; i >= 0; --i) { /* 32-bit limb 7 - i from the bottom */
    uint64_t t = (uint64_t)w[i] * m + carry;
    int limb = 7 - i;
    Q[limb / 2] |= (uint64_t)(uint32_t)t << (32 * (limb % 2));
    carry = t >> 32;
  }
  Q[4] = carry;
  int F = 255 - E + s; /* bits >= F form the integer part */
  int q = (int)(get64n(Q, 5, F) & 3u);
  unsigned __int128 fr = ((unsigned __int128)get64n(Q, 5, F - 64) << 64) | get64n(Q, 5, F - 128);
  __int128 sf;
  if (fr >> 127) { /* f >= 1/2: take f - 1 and the next integer */
    sf = (__int128)(fr - ((unsigned __int128)1 << 127)) - ((__int128)1 << 127);
    q += 1;
  } else {
    sf = (__int128)fr;
  }
  *quadrant = q & 3;
  double hi = (double)sf;
  double lo = (double)(sf - (__int128)hi);
  return fast_two_sum(ldexp(hi, -128), ldexp(lo, -128));
}

/* ---- the functions: pair values ---------------------------------------- */

/* returns 0 and a pair for finite results that need rounding; 1 with *rn
   set for exact or special results.  kind: 0 sin, 1 cos, 2 tan */
static int trig_value(float x, int kind, dd* v, float* rn) {
  if (isnan(x) || isinf(x)) {
    *rn = NAN;
    return 1;
  }
  if (x == 0.0f) {
    *rn = kind == 1 ? 1.0f : x;
    return 1;
  }
  double ax = fabs((double)x);
  dd r;
  int k;
  if (ax < 0.78539816339744830) { /* below pi/4 */
    r = dd_from(ax);
    k = 0;
  } else {
    int e;
    double mant = frexp(ax, &e); /* ax = mant 2^e, mant in [0.5, 1) */
    uint32_t m = (uint32_t)ldexp(mant, 24);
    dd f = reduce_2_over_pi(m, e - 24, &k);
    r = dd_mul(f, (dd){PIO2_D[0], PIO2_D[1]});
  }
  /* |x| = k pi/2 + r */
  dd s;
  if (kind == 2) {
    dd sn = sin_series(r), cs = cos_series(r);
    s = (k & 1) ? dd_neg(dd_div(cs, sn)) : dd_div(sn, cs);
  } else {
    int q = (k + kind) & 3; /* cos |x| = sin(|x| + pi/2) */
    s = (q & 1) ? cos_series(r) : sin_series(r);
    if (q & 2) s = dd_neg(s);
  }
  if (x < 0.0f && kind != 1) s = dd_neg(s); /* sin and tan are odd, cos even */
  *v = s;
  return 0;
}

static int exp_value(float x, dd* v, float* rn) {
  if (isnan(x)) {
    *rn = x;
    return 1;
  }
  if (x == 0.0f) {
    *rn = 1.0f;
    return 1;
  }
  if (x > 89.0f) { /* e^89 > 2^128 */
    *rn = INFINITY;
    return 1;
  }
  if (x < -104.0f) { /* e^-104 < 2^-150: rounds to +0 */
    *rn = 0.0f;
    return 1;
  }
  double xd = (double)x;
  double k = nearbyint(xd / LN2_D[0]);
  /* r = x - k (l0 + l1 + l2): k l0 is not exact in general; use the pair
     products and exact sums */
  dd p0 = two_prod(k, LN2_D[0]);
  dd p1 = two_prod(k, LN2_D[1]);
  dd r = dd_add(dd_from(xd), dd_neg(p0));
  r = dd_add(r, dd_neg(p1));
  r = dd_add(r, dd_from(-k * LN2_D[2]));
  dd e = exp_series(r);
  e.hi = ldexp(e.hi, (int)k);
  e.lo = ldexp(e.lo, (int)k);
  *v = e;
  return 0;
}

static int log_value(float x, dd* v, float* rn) {
  if (isnan(x)) {
    *rn = x;
    return 1;
  }
  if (x < 0.0f) {
    *rn = NAN;
    return 1;
  }
  if (x == 0.0f) {
    *rn = -INFINITY;
    return 1;
  }
  if (isinf(x)) {
    *rn = x;
    return 1;
  }
  if (x == 1.0f) {
    *rn = 0.0f;
    return 1;
  }
  int e;
  double m = frexp((double)x, &e); /* [0.5, 1) */
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  /* t = (m - 1)/(m + 1): m - 1 and m + 1 are exact (m has 24 bits) */
  dd t = dd_div(dd_from(m - 1.0), dd_from(m + 1.0));
  dd l = atanh2_series(t);
  dd el = dd_add(two_prod((double)e, LN2_D[0]), two_prod((double)e, LN2_D[1]));
  el = dd_add(el, dd_from((double)e * LN2_D[2]));
  *v = dd_add(el, l);
  return 0;
}

static int exp2_value(float x, dd* v, float* rn) {
  if (isnan(x)) {
    *rn = x;
    return 1;
  }
  if (x > 128.5f) {
    *rn = INFINITY;
    return 1;
  }
  if (x < -151.0f) {
    *rn = 0.0f;
    return 1;
  }
  double xd = (double)x;
  double k = nearbyint(xd);
  if (xd == k) { /* exact powers of two */
    *rn = (float)ldexp(1.0, (int)k);
    return 1;
  }
  /* 2^f = e^(f ln 2), f = x - k exact, |f ln2| <= 0.35 */
  dd a = dd_mul_d((dd){LN2_D[0], LN2_D[1]}, xd - k);
  dd e = exp_series(a);
  e.hi = ldexp(e.hi, (int)k);
  e.lo = ldexp(e.lo, (int)k);
  *v = e;
  return 0;
}

static int log2_value(float x, dd* v, float* rn) {
  int special = log_value(x, v, rn);
  if (special) return 1;
  int e;
  double m = frexp((double)x, &e);
  if (m == 0.5) { /* powers of two: exact */
    *rn = (float)(e - 1);
    return 1;
  }
  *v = dd_mul(*v, INV_LN2);
  return 0;
}

static int hyp_value(float x, int kind, dd* v, float* rn) { /* 0 sinh, 1 cosh, 2 tanh */
  if (isnan(x)) {
    *rn = x;
    return 1;
  }
  double ax = fabs((double)x);
  if (x == 0.0f) {
    *rn = kind == 1 ? 1.0f : x;
    return 1;
  }
  if (kind == 2 && ax > 20.0) { /* tanh = 1 - 2 e^(-2|x|) + ...: the pair (1, -2 e^(-2|x|)) */
    dd t = {1.0, -2.0 * exp(-2.0 * ax)};
    *v = x < 0.0f ? dd_neg(t) : t;
    return 0;
  }
  if (kind != 2 && ax > 90.0) { /* e^90 / 2 > 2^128 */
    *rn = kind == 1 ? INFINITY : copysignf(INFINITY, x);
    return 1;
  }
  dd s;
  if (kind != 1 && ax < 0.0625) {
    dd sh = sinh_small(dd_from(ax));
    if (kind == 0) {
      s = sh;
    } else { /* tanh = sinh / sqrt(1 + sinh^2) */
      dd one = dd_add(dd_from(1.0), dd_mul(sh, sh));
      double r0 = sqrt(one.hi);
      dd q = dd_add(one, dd_neg(two_prod(r0, r0)));
      dd root = dd_add(dd_from(r0), dd_from(q.hi / (2.0 * r0)));
      s = dd_div(sh, root);
    }
  } else {
    dd E = exp_pair(ax);
    dd iE = dd_div(dd_from(1.0), E);
    if (kind == 0) {
      s = dd_add(E, dd_neg(iE));
    } else if (kind == 1) {
      s = dd_add(E, iE);
    } else {
      s = dd_div(dd_add(E, dd_neg(iE)), dd_add(E, iE));
    }
    if (kind != 2) {
      s.hi *= 0.5;
      s.lo *= 0.5;
    }
  }
  if (x < 0.0f && kind != 1) s = dd_neg(s);
  *v = s;
  return 0;
}

/* ---- rounding to binary32 ----------------------------------------------- */

/* distance |v - c| for a float candidate c (c = 2^128 stands for +inf) */
static double dist(dd v, double c) {
  dd d = two_sum(v.hi, -c);
  return fabs(d.hi + (d.lo + v.lo));
}

/* correctly rounded binary32 value of v, given |v - exact| <= rel |exact|;
   returns 1 if the bound does not decide it */
static int round_f32(dd v, double rel, float* out) {
  double a = fabs(v.hi);
  double tol = rel * a * 1.01 + 0x1p-300;
  float f = (float)v.hi;
  double cands[3];
  float fl[3];
  if (isinf(f)) {
    fl[0] = copysignf(INFINITY, f);
    cands[0] = copysign(0x1p128, v.hi);
    fl[1] = copysignf(0x1.fffffep127f, f);
    cands[1] = (double)fl[1];
    fl[2] = fl[1];
    cands[2] = cands[1];
  } else {
    fl[0] = f;
    fl[1] = nextafterf(f, -INFINITY);
    fl[2] = nextafterf(f, INFINITY);
    for (int i = 0; i < 3; ++i) cands[i] = isinf(fl[i]) ? copysign(0x1p128, (double)fl[i]) : (double)fl[i];
  }
  double d[3];
  for (int i = 0; i < 3; ++i) d[i] = dist(v, cands[i]);
  int best = 0;
  for (int i = 1; i < 3; ++i)
    if (d[i] < d[best]) best = i;
  double second = INFINITY;
  for (int i = 0; i < 3; ++i)
    if (i != best && fl[i] != fl[best] && d[i] < second) second = d[i];
  *out = fl[best];
  /* undecided when the two nearest candidates are within the error of
     being equally near */
  return second - d[best] <= 2.0 * tol;
}

/* ---- exported entry points ---------------------------------------------- */

enum { FN_SIN, FN_EXP, FN_LOG, FN_COS, FN_TAN, FN_EXP2, FN_LOG2, FN_SINH, FN_COSH, FN_TANH,
       FN_ASIN, FN_ACOS, FN_ATAN, FN_LOG10, FN_LOG1P, FN_EXP10, FN_EXPM1, FN_CBRT, FN_ASINH,
       FN_ACOSH, FN_ATANH, FN_ERF, FN_ERFC, FN_LGAMMA, FN_TGAMMA };

/* the cores of binary.h for a binary32 argument, unscaled (binary32
   results that neither overflow nor round to zero lie in the binary64
   normal range) */
static int inv_value(int fn, float x, dd* v, float* rn) {
  int k;
  double r;
  int sp;
  switch (fn) {
    case FN_ASIN: sp = asin_core(x, v, &k, &r); break;
    case FN_ACOS: sp = acos_core(x, v, &k, &r); break;
    case FN_ATAN: sp = atan_core(x, v, &k, &r); break;
    case FN_LOG10: sp = log10_core(x, v, &k, &r); break;
    case FN_LOG1P: sp = log1p_core(x, v, &k, &r); break;
    case FN_EXP10: sp = exp10_core(x, 89.5, -104.5, v, &k, &r); break;
    case FN_EXPM1: sp = expm1_core(x, 89.5, v, &k, &r); break;
    case FN_ASINH: sp = asinh_core(x, v, &k, &r); break;
    case FN_ACOSH: sp = acosh_core(x, v, &k, &r); break;
    case FN_ATANH: sp = atanh_core(x, v, &k, &r); break;
    case FN_ERF: sp = erf_core(x, v, &k, &r); break;
    case FN_ERFC: sp = erfc_core(x, v, &k, &r); break;
    default: sp = cbrt_core(x, v, &k, &r); break;
  }
  if (sp) {
    *rn = (float)r;
    return 1;
  }
  v->hi = ldexp(v->hi, k);
  v->lo = ldexp(v->lo, k);
  return 0;
}

static const double REL = 0x1p-90;

/* lgamma and tgamma, unscaled, with their own relative bound *rel */
static int gamma_value(int fn, float x, dd* v, float* rn, double* rel) {
  double r;
  int k = 0;
  int sp = fn == FN_LGAMMA ? lgamma_core(x, v, &k, rel, &r)
                           : tgamma_core(x, 89.5, -104.5, v, &k, rel, &r);
  if (sp) {
    *rn = (float)r;
    return 1;
  }
  v->hi = ldexp(v->hi, k);
  v->lo = ldexp(v->lo, k);
  return 0;
}

/* the value of fn at x: 1 with *rn for an exact result, else 0 with the
   pair v and its relative error bound *rel */
static int value(int fn, float x, dd* v, float* rn, double* rel) {
  *rel = REL;
  switch (fn) {
    case FN_LGAMMA:
    case FN_TGAMMA: return gamma_value(fn, x, v, rn, rel);
    case FN_ASIN:
    case FN_ACOS:
    case FN_ATAN:
    case FN_LOG10:
    case FN_LOG1P:
    case FN_EXP10:
    case FN_EXPM1:
    case FN_CBRT:
    case FN_ASINH:
    case FN_ACOSH:
    case FN_ATANH:
    case FN_ERF:
    case FN_ERFC: return inv_value(fn, x, v, rn);
    case FN_SIN: return trig_value(x, 0, v, rn);
    case FN_COS: return trig_value(x, 1, v, rn);
    case FN_TAN: return trig_value(x, 2, v, rn);
    case FN_EXP: return exp_value(x, v, rn);
    case FN_EXP2: return exp2_value(x, v, rn);
    case FN_LOG: return log_value(x, v, rn);
    case FN_LOG2: return log2_value(x, v, rn);
    case FN_SINH: return hyp_value(x, 0, v, rn);
    case FN_COSH: return hyp_value(x, 1, v, rn);
    default: return hyp_value(x, 2, v, rn);
  }
}

/* n inputs: hi/lo the pair (NaN for special results), rn the rounded value,
   undecided[i] = 1 where the caller must ask the ball oracle */
void oracle_fast32_eval(int fn, const float* x, long n, double* hi, double* lo, float* rn,
                        uint8_t* undecided) {
  for (long i = 0; i < n; ++i) {
    dd v;
    float r;
    double rel;
    if (value(fn, x[i], &v, &r, &rel)) {
      hi[i] = (double)r;
      lo[i] = 0.0;
      rn[i] = r;
      undecided[i] = 0;
      continue;
    }
    undecided[i] = (uint8_t)round_f32(v, rel, &r);
    hi[i] = v.hi;
    lo[i] = v.lo;
    rn[i] = r;
  }
}

/* the relative error bound the stage claims for each input's pair (0 for
   the exact results) */
void oracle_fast32_rel(int fn, const float* x, long n, double* rel) {
  for (long i = 0; i < n; ++i) {
    dd v;
    float r;
    rel[i] = value(fn, x[i], &v, &r, &rel[i]) ? 0.0 : rel[i];
  }
}

static inline float from_bits(uint32_t b) {
  float f;
  memcpy(&f, &b, 4);
  return f;
}

static inline uint32_t bits_of(float f) {
  uint32_t b;
  memcpy(&b, &f, 4);
  return b;
}

/* the host libm's binary64 function */
static double libm_double(int fn, double d) {
  switch (fn) {
    case FN_SIN: return sin(d);
    case FN_COS: return cos(d);
    case FN_TAN: return tan(d);
    case FN_EXP: return exp(d);
    case FN_EXP2: return exp2(d);
    case FN_LOG: return log(d);
    case FN_LOG2: return log2(d);
    case FN_SINH: return sinh(d);
    case FN_COSH: return cosh(d);
    case FN_ASIN: return asin(d);
    case FN_ACOS: return acos(d);
    case FN_ATAN: return atan(d);
    case FN_LOG10: return log10(d);
    case FN_LOG1P: return log1p(d);
    case FN_EXP10: return exp10(d);
    case FN_EXPM1: return expm1(d);
    case FN_CBRT: return cbrt(d);
    case FN_ASINH: return asinh(d);
    case FN_ACOSH: return acosh(d);
    case FN_ATANH: return atanh(d);
    case FN_ERF: return erf(d);
    case FN_ERFC: return erfc(d);
    case FN_LGAMMA: return lgamma(d);
    case FN_TGAMMA: return tgamma(d);
    default: return tanh(d);
  }
}

typedef struct {
  long n, undecided, differ, differ_explained;
} sweep_stats;

/* every bit pattern in [start, start + count): the oracle against glibc's
   binary64 result rounded to binary32.  Where the two differ, the binary64
   result should lie within two of its own ulps of a binary32 midpoint (a
   double rounding); those are counted as explained.  Inputs that differ or
   are undecided are stored (up to cap each) for the ball oracle. */
void oracle_fast32_sweep_libm(int fn, uint64_t start, uint64_t count, sweep_stats* st,
                              uint32_t* differ, long differ_cap, uint32_t* undec, long undec_cap) {
  memset(st, 0, sizeof(*st));
  for (uint64_t i = 0; i < count; ++i) {
    uint32_t b = (uint32_t)(start + i);
    float x = from_bits(b);
    dd v;
    float r;
    double rel;
    st->n++;
    if (!value(fn, x, &v, &r, &rel)) {
      if (round_f32(v, rel, &r)) {
        if (st->undecided < undec_cap) undec[st->undecided] = b;
        st->undecided++;
        continue;
      }
    }
    double d = libm_double(fn, (double)x);
    float g = (float)d;
    int same = (bits_of(g) == bits_of(r)) || (isnan(g) && isnan(r));
    if (!same) {
      if (st->differ < differ_cap) differ[st->differ] = b;
      st->differ++;
      /* the binary32 midpoint between r and g */
      double mid = 0.5 * ((double)r + (double)g);
      double ulp_d = fabs(nextafter(d, INFINITY) - d);
      if (!isinf(g) && !isinf(r) && fabs(d - mid) <= 2.0 * ulp_d) st->differ_explained++;
    }
  }
}

typedef struct {
  long n, undecided, special_mismatch, violations;
  double max_ulp, sum_ulp;
  long n_reg;
  uint32_t worst;
} check_stats;

/* GPU results y for the bit patterns [start, start + count) against the
   oracle, with the ULP metric of tests/ulp.py: ulp(v) = 2^(max(floor(log2
   |v|), -126) - 23) at the exact value v; NaN, +-inf, +-0 and subnormal
   correctly rounded results must match bit for bit (NaN as a class). */
/* one result y of input x into the statistics (the ULP metric of
   tests/ulp.py); returns 1 for an undecided input, 2 for a failure */
static int check_value(int exact, dd v, float r, double rel, float x, float yi, double bound,
                       check_stats* st);

static int check_one(int fn, float x, float yi, double bound, check_stats* st) {
  dd v;
  float r;
  double rel;
  int exact = value(fn, x, &v, &r, &rel);
  return check_value(exact, v, r, rel, x, yi, bound, st);
}

/* one result yi against the value v (or the exact r): 0 fine, 1 undecided,
   2 outside the bound or a special mismatch */
static int check_value(int exact, dd v, float r, double rel, float x, float yi, double bound,
                       check_stats* st) {
  st->n++;
  if (exact) {
    v.hi = (double)r; /* an exact result: the pair is the value itself */
    v.lo = 0.0;
  } else if (round_f32(v, rel, &r)) {
    st->undecided++;
    return 1;
  }
  int same = (bits_of(yi) == bits_of(r)) || (isnan(yi) && isnan(r));
  if (isnan(r) || isinf(r) || r == 0.0f || fabsf(r) < 0x1p-126f) {
    if (!same) {
      st->special_mismatch++;
      return 2;
    }
    return 0;
  }
  double av = fabs(v.hi);
  int e;
  frexp(av, &e);
  e -= 1; /* floor(log2 |hi|) */
  if (av == ldexp(1.0, e) && v.lo != 0.0 && (v.lo < 0) != (v.hi < 0)) e -= 1;
  if (e < -126) e = -126;
  double ulp = ldexp(1.0, e - 23);
  double err;
  if (isnan(yi)) {
    err = INFINITY;
  } else if (isinf(yi)) {
    err = fabs((copysign(0x1p127, (double)yi) - 0.5 * v.hi) - 0.5 * v.lo) / (0.5 * ulp);
  } else {
    err = fabs(((double)yi - v.hi) - v.lo) / ulp;
  }
  if (same && err > 0.5) err = 0.5;
  st->n_reg++;
  st->sum_ulp += err;
  if (err > st->max_ulp) {
    st->max_ulp = err;
    st->worst = bits_of(x);
  }
  if (err > bound) {
    st->violations++;
    return 2;
  }
  return 0;
}

/* GPU results y for the bit patterns [start, start + count) against the
   oracle: NaN, +-inf, +-0 and subnormal correctly rounded results bit for
   bit (NaN as a class), the others within bound ULP (ulp(v) = 2^(max(floor(
   log2 |v|), -126) - 23) at the exact value v). */
void oracle_fast32_check(int fn, uint64_t start, uint64_t count, const float* y, double bound,
                         check_stats* st, uint32_t* bad, long bad_cap, uint32_t* undec,
                         long undec_cap) {
  memset(st, 0, sizeof(*st));
  long nb = 0, nu = 0;
  for (uint64_t i = 0; i < count; ++i) {
    uint32_t b = (uint32_t)(start + i);
    int c = check_one(fn, from_bits(b), y[i], bound, st);
    if (c == 1 && nu < undec_cap) undec[nu++] = b;
    if (c == 2 && nb < bad_cap) bad[nb++] = b;
  }
}

/* the same for arbitrary inputs x (indices of failures and undecided ones) */
void oracle_fast32_check_x(int fn, const float* x, const float* y, long n, double bound,
                           check_stats* st, long* bad, long bad_cap, long* undec, long undec_cap) {
  memset(st, 0, sizeof(*st));
  long nb = 0, nu = 0;
  for (long i = 0; i < n; ++i) {
    int c = check_one(fn, x[i], y[i], bound, st);
    if (c == 1 && nu < undec_cap) undec[nu++] = i;
    if (c == 2 && nb < bad_cap) bad[nb++] = i;
  }
}

/* ---- pow and atan2 ----------------------------------------------------------- */

enum { B_POW, B_ATAN2 };
static const double REL_POW = 0x1p-86, REL_ATAN2 = 0x1p-90;

/* the value for binary32 operands, unscaled (every such result that does
   not round to 0 or overflow lies in the binary64 normal range) */
static int value2(int fn, float a, float b, dd* v, float* rn) {
  int k;
  double r;
  int sp = fn == B_POW ? pow_core(a, b, 89.5, -104.5, v, &k, &r) : atan2_core(a, b, v, &k, &r);
  if (sp) {
    *rn = (float)r;
    return 1;
  }
  v->hi = ldexp(v->hi, k);
  v->lo = ldexp(v->lo, k);
  return 0;
}

void oracle_fast32_eval2(int fn, const float* a, const float* b, long n, double* hi, double* lo,
                         float* rn, uint8_t* undecided) {
  double rel = fn == B_POW ? REL_POW : REL_ATAN2;
  for (long i = 0; i < n; ++i) {
    dd v;
    float r;
    if (value2(fn, a[i], b[i], &v, &r)) {
      hi[i] = (double)r;
      lo[i] = 0.0;
      rn[i] = r;
      undecided[i] = 0;
      continue;
    }
    undecided[i] = (uint8_t)round_f32(v, rel, &r);
    hi[i] = v.hi;
    lo[i] = v.lo;
    rn[i] = r;
  }
}

void oracle_fast32_check2(int fn, const float* a, const float* b, const float* y, long n,
                          double bound, check_stats* st, long* bad, long bad_cap, long* undec,
                          long undec_cap) {
  memset(st, 0, sizeof(*st));
  double rel = fn == B_POW ? REL_POW : REL_ATAN2;
  long nb = 0, nu = 0;
  for (long i = 0; i < n; ++i) {
    dd v;
    float r;
    int exact = value2(fn, a[i], b[i], &v, &r);
    int c = check_value(exact, v, r, rel, a[i], y[i], bound, st);
    if (c == 1 && nu < undec_cap) undec[nu++] = i;
    if (c == 2 && nb < bad_cap) bad[nb++] = i;
  }
}
