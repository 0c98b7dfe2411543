/* Fast first stage of the oracle for binary64 sin, cos, tan, exp, exp2, log,
 * log2, sinh, cosh and tanh.
 *
 * TEST INFRASTRUCTURE ONLY (see fast32.c): the same methods as the binary32
 * stage, sized for 53-bit inputs.  Each value is a double-double v times
 * 2^k (k keeps results near and below the binary64 range exact) with
 * |v 2^k - f(x)| <= 2^-90 |f(x)| (checked in tests/test_oracle_fast.py
 * against mpmath); the correctly rounded binary64 result is returned where
 * that bound decides it, else the input is reported undecided and the ball
 * oracle answers.
 *
 *  sin, cos, tan: 2|x|/pi = q + f from the exact product of the 53-bit
 *       mantissa with 320 bits of 2/pi (192 fraction bits kept: the smallest
 *       reduced argument of a binary64 input is about 2^-62 of pi/2, so f
 *       keeps at least 130 significant bits), r = f pi/2, Taylor series.
 *  exp, exp2: k ln 2 (three doubles) or the nearest integer, Taylor series
 *       of e^r, the power of two kept apart.
 *  log, log2: 2 atanh((m - 1)/(m + 1)) for m in [1/sqrt 2, sqrt 2) (m + 1 as
 *       an exact pair) plus e ln 2; log2 = log / ln 2, powers of two exact.
 *  sinh, cosh, tanh: from e^|x| and its reciprocal below |x| = 40, Taylor
 *       below 2^-4 (sinh, tanh), e^|x| / 2 and 1 - 2 e^(-2|x|) above 40.
 */
#include "binary.h"

/* |x| = m 2^E (m < 2^53 an integer): 2|x|/pi = q + f, q modulo 4, |f| <= 1/2
   as a pair (relative error below 2^-120) */
static dd reduce64(uint64_t m, int E, int* quadrant) {
  int s = E - 1 > 1 ? E - 1 : 1;
  uint32_t w[10];
  for (int i = 0; i < 10; ++i) w[i] = tbits32(s - 1 + 32 * i);
  uint64_t W[5];
  for (int k = 0; k < 5; ++k) W[k] = ((uint64_t)w[8 - 2 * k] << 32) | w[9 - 2 * k];
  /* P = m W (373 bits, little-endian 64-bit words); value = P 2^(E - s - 319) */
  uint64_t P[6];
  unsigned __int128 carry = 0;
  for (int k = 0; k < 5; ++k) {
    unsigned __int128 t = (unsigned __int128)W[k] * m + carry;
    P[k] = (uint64_t)t;
    carry = t >> 64;
  }
  P[5] = (uint64_t)carry;
  int F = s + 319 - E; /* bits >= F form the integer part */
  int q = (int)(get64n(P, 6, F) & 3u);
  /* 192 fraction bits, most significant word first */
  uint64_t f2 = get64n(P, 6, F - 64), f1 = get64n(P, 6, F - 128), f0 = get64n(P, 6, F - 192);
  int neg = (int)(f2 >> 63);
  if (neg) { /* f >= 1/2: f - 1 = -(2^192 - fraction) / 2^192, and the next integer */
    q += 1;
    f0 = ~f0;
    f1 = ~f1;
    f2 = ~f2;
    if (++f0 == 0 && ++f1 == 0) ++f2;
  }
  *quadrant = q & 3;
  /* normalise the 192-bit magnitude and keep its top 128 bits */
  int lz = 0;
  uint64_t a = f2, b = f1, c = f0;
  while (a == 0 && lz < 192) {
    a = b;
    b = c;
    c = 0;
    lz += 64;
  }
  if (a == 0) return dd_from(0.0);
  int sh = __builtin_clzll(a);
  if (sh) {
    a = (a << sh) | (b >> (64 - sh));
    b = (b << sh) | (c >> (64 - sh));
  }
  lz += sh;
  /* the top 127 bits, so that the rounded double stays below 2^127 */
  unsigned __int128 top = (((unsigned __int128)a << 64) | b) >> 1;
  double hi = (double)top;
  double lo = (double)(__int128)(top - (unsigned __int128)hi);
  /* f = top 2^-(127 + lz) */
  dd f = fast_two_sum(ldexp(hi, -127 - lz), ldexp(lo, -127 - lz));
  return neg ? dd_neg(f) : f;
}

/* ---- values: v 2^k, or an exact / special result in *rn ----------------- */

static int trig64(double x, int kind, dd* v, int* k, double* rn) {
  *k = 0;
  if (isnan(x) || isinf(x)) {
    *rn = NAN;
    return 1;
  }
  if (x == 0.0) {
    *rn = kind == 1 ? 1.0 : x;
    return 1;
  }
  double ax = fabs(x);
  dd r;
  int q;
  if (ax < 0.78539816339744830) {
    r = dd_from(ax);
    q = 0;
  } else {
    int e;
    double mant = frexp(ax, &e);
    uint64_t m = (uint64_t)ldexp(mant, 53);
    dd f = reduce64(m, e - 53, &q);
    r = dd_mul(f, (dd){PIO2_D[0], PIO2_D[1]});
  }
  dd s;
  if (kind == 2) {
    dd sn = sin_series(r), cs = cos_series(r);
    s = (q & 1) ? dd_neg(dd_div(cs, sn)) : dd_div(sn, cs);
  } else {
    int qq = (q + kind) & 3;
    s = (qq & 1) ? cos_series(r) : sin_series(r);
    if (qq & 2) s = dd_neg(s);
  }
  if (x < 0.0 && kind != 1) s = dd_neg(s);
  *v = s;
  return 0;
}

static int exp64(double x, int base2, dd* v, int* k, double* rn) {
  *k = 0;
  if (isnan(x)) {
    *rn = x;
    return 1;
  }
  double hi_lim = base2 ? 1025.0 : 710.0, lo_lim = base2 ? -1076.0 : -746.0;
  if (x > hi_lim) {
    *rn = INFINITY;
    return 1;
  }
  if (x < lo_lim) {
    *rn = 0.0;
    return 1;
  }
  if (x == 0.0) {
    *rn = 1.0;
    return 1;
  }
  if (base2) {
    double kk = nearbyint(x);
    if (kk == x) {
      *rn = ldexp(1.0, (int)kk);
      return 1;
    }
    *v = exp_series(dd_mul_d((dd){LN2_D[0], LN2_D[1]}, x - kk));
    *k = (int)kk;
    return 0;
  }
  double kk = nearbyint(x / LN2_D[0]);
  dd r = dd_add(dd_from(x), dd_neg(two_prod(kk, LN2_D[0])));
  r = dd_add(r, dd_neg(two_prod(kk, LN2_D[1])));
  r = dd_add(r, dd_from(-kk * LN2_D[2]));
  *v = exp_series(r);
  *k = (int)kk;
  return 0;
}

static int log64(double x, int base2, dd* v, int* k, double* rn) {
  *k = 0;
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
  int e;
  double m = frexp(x, &e);
  if (m == 0.5) { /* powers of two */
    if (base2) {
      *rn = (double)(e - 1);
      return 1;
    }
    if (e == 1) {
      *rn = 0.0;
      return 1;
    }
  }
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  dd t = dd_div(dd_from(m - 1.0), two_sum(m, 1.0));
  dd l = atanh2_series(t);
  dd el = dd_add(two_prod((double)e, LN2_D[0]), two_prod((double)e, LN2_D[1]));
  el = dd_add(el, dd_from((double)e * LN2_D[2]));
  dd s = dd_add(el, l);
  *v = base2 ? dd_mul(s, INV_LN2) : s;
  return 0;
}

static int hyp64(double x, int kind, dd* v, int* k, double* rn) {
  *k = 0;
  if (isnan(x)) {
    *rn = x;
    return 1;
  }
  if (x == 0.0) {
    *rn = kind == 1 ? 1.0 : x;
    return 1;
  }
  double ax = fabs(x);
  dd s;
  if (ax > 40.0) { /* e^-2|x| < 2^-115 of the result */
    if (kind == 2) {
      s = (dd){1.0, -2.0 * exp(-2.0 * ax)};
    } else {
      if (ax > 711.0) {
        *rn = kind == 1 ? INFINITY : copysign(INFINITY, x);
        return 1;
      }
      double kk = nearbyint(ax / LN2_D[0]);
      dd r = dd_add(dd_from(ax), dd_neg(two_prod(kk, LN2_D[0])));
      r = dd_add(r, dd_neg(two_prod(kk, LN2_D[1])));
      r = dd_add(r, dd_from(-kk * LN2_D[2]));
      s = exp_series(r);
      *k = (int)kk - 1;
    }
  } else if (kind != 1 && ax < 0.0625) {
    dd sh = sinh_small(dd_from(ax));
    if (kind == 0) {
      s = sh;
    } else {
      dd one = dd_add(dd_from(1.0), dd_mul(sh, sh));
      double r0 = sqrt(one.hi);
      dd qq = dd_add(one, dd_neg(two_prod(r0, r0)));
      dd root = dd_add(dd_from(r0), dd_from(qq.hi / (2.0 * r0)));
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
  if (x < 0.0 && kind != 1) s = dd_neg(s);
  *v = s;
  return 0;
}

enum { G_SIN, G_EXP, G_LOG, G_COS, G_TAN, G_EXP2, G_LOG2, G_SINH, G_COSH, G_TANH, G_ASIN,
       G_ACOS, G_ATAN, G_LOG10, G_LOG1P, G_EXP10, G_EXPM1, G_CBRT, G_ASINH, G_ACOSH, G_ATANH,
       G_ERF, G_ERFC, G_LGAMMA, G_TGAMMA };

static const double REL64 = 0x1p-90;

/* the value of fn at x: 1 with *rn for an exact result, else 0 with v 2^k
   and *rel, the relative error bound of v (2^-90 but for lgamma and tgamma,
   which carry their own) */
static int value64(int fn, double x, dd* v, int* k, double* rn, double* rel) {
  *rel = REL64;
  switch (fn) {
    case G_LGAMMA: return lgamma_core(x, v, k, rel, rn);
    case G_TGAMMA: return tgamma_core(x, 710.5, -746.5, v, k, rel, rn);
    case G_ASIN: return asin_core(x, v, k, rn);
    case G_ACOS: return acos_core(x, v, k, rn);
    case G_ATAN: return atan_core(x, v, k, rn);
    case G_LOG10: return log10_core(x, v, k, rn);
    case G_LOG1P: return log1p_core(x, v, k, rn);
    case G_EXP10: return exp10_core(x, 710.5, -746.5, v, k, rn);
    case G_EXPM1: return expm1_core(x, 710.5, v, k, rn);
    case G_CBRT: return cbrt_core(x, v, k, rn);
    case G_ASINH: return asinh_core(x, v, k, rn);
    case G_ACOSH: return acosh_core(x, v, k, rn);
    case G_ATANH: return atanh_core(x, v, k, rn);
    case G_ERF: return erf_core(x, v, k, rn);
    case G_ERFC: return erfc_core(x, v, k, rn);
    case G_SIN: return trig64(x, 0, v, k, rn);
    case G_COS: return trig64(x, 1, v, k, rn);
    case G_TAN: return trig64(x, 2, v, k, rn);
    case G_EXP: return exp64(x, 0, v, k, rn);
    case G_EXP2: return exp64(x, 1, v, k, rn);
    case G_LOG: return log64(x, 0, v, k, rn);
    case G_LOG2: return log64(x, 1, v, k, rn);
    case G_SINH: return hyp64(x, 0, v, k, rn);
    case G_COSH: return hyp64(x, 1, v, k, rn);
    default: return hyp64(x, 2, v, k, rn);
  }
}

/* ---- rounding v 2^k to binary64 ----------------------------------------- */

static int round_f64(dd v, int k, double rel, double* out) {
  v = fast_two_sum(v.hi, v.lo);
  if (v.hi == 0.0) {
    *out = v.hi;
    return 0;
  }
  int e;
  frexp(v.hi, &e);
  int E = e - 1 + k; /* about floor(log2 |value|) */
  double tol = rel * fabs(v.hi) * 1.01;
  if (E >= -1021) { /* normal (or overflowing) results */
    double f = v.hi + v.lo; /* the pair rounded to 53 bits */
    int ef;
    frexp(f, &ef);
    double u = ldexp(1.0, ef - 53); /* ulp of f */
    double d = (v.hi - f) + v.lo;
    int undecided = fabs(fabs(d) - 0.5 * u) <= tol;
    if (fabs(f) == ldexp(1.0, ef - 1) && (d < 0) == (f > 0)) /* below a power of two */
      undecided |= fabs(fabs(d) - 0.25 * u) <= tol;
    *out = ldexp(f, k);
    return undecided;
  }
  /* subnormal range: units of 2^-1074 */
  double h = ldexp(v.hi, k + 1074), l = ldexp(v.lo, k + 1074);
  double n = nearbyint(h);
  double d = (h - n) + l;
  double tu = rel * fabs(h) * 1.01 + 0x1p-60;
  int undecided = fabs(fabs(d) - 0.5) <= tu;
  n = d > 0.5 ? n + 1.0 : (d < -0.5 ? n - 1.0 : n);
  *out = ldexp(n, -1074);
  if (*out == 0.0) *out = copysign(0.0, v.hi);
  return undecided;
}

/* n inputs: rn the correctly rounded result, hi/lo the value as a pair
   (scaled, so rounded near the bottom of the range), undecided[i] = 1 where
   the ball oracle must answer */
void oracle_fast64_eval(int fn, const double* x, long n, double* hi, double* lo, double* rn,
                        uint8_t* undecided) {
  for (long i = 0; i < n; ++i) {
    dd v;
    int k;
    double r, rel;
    if (value64(fn, x[i], &v, &k, &r, &rel)) {
      hi[i] = r;
      lo[i] = 0.0;
      rn[i] = r;
      undecided[i] = 0;
      continue;
    }
    undecided[i] = (uint8_t)round_f64(v, k, rel, &r);
    hi[i] = ldexp(v.hi, k);
    lo[i] = ldexp(v.lo, k);
    rn[i] = r;
  }
}

static inline uint64_t bits64(double f) {
  uint64_t b;
  memcpy(&b, &f, 8);
  return b;
}

typedef struct {
  long n, undecided, special_mismatch, violations;
  double max_ulp, sum_ulp;
  long n_reg;
  long worst;
} check64_stats;

/* results y of inputs x against the oracle, the ULP metric of tests/ulp.py
   in binary64 (ulp(v) = 2^(max(floor(log2 |v|), -1022) - 52)); NaN, +-inf,
   +-0 and subnormal correctly rounded results bit for bit (NaN as a class).
   Undecided inputs are listed (their indices) for the ball oracle. */
/* one result yi against the value v 2^k (or the exact r): 0 fine, 1
   undecided (the ball oracle must answer), 2 outside the bound or a special
   mismatch */
static int check_elem(int exact, dd v, int k, double r, double rel, double yi, double bound,
                      check64_stats* st, long i) {
  st->n++;
  if (exact) {
    v = dd_from(r);
    k = 0;
  } else if (round_f64(v, k, rel, &r)) {
    st->undecided++;
    return 1;
  }
  int same = (bits64(yi) == bits64(r)) || (isnan(yi) && isnan(r));
  if (isnan(r) || isinf(r) || r == 0.0 || fabs(r) < 0x1p-1022) {
    if (!same) {
      st->special_mismatch++;
      return 2;
    }
    return 0;
  }
  /* floor(log2 |value|), the pair scaled by 2^k */
  int e;
  frexp(v.hi, &e);
  int E = e - 1 + k;
  if (fabs(v.hi) == ldexp(1.0, e - 1) && v.lo != 0.0 && (v.lo < 0) != (v.hi < 0)) E -= 1;
  if (E < -1022) E = -1022;
  /* error in ulps, computed in the scaled domain */
  double err;
  if (isnan(yi)) {
    err = INFINITY;
  } else if (isinf(yi)) {
    /* 2^1024 against the value, halved to stay finite */
    double yh = copysign(0x1p1023, yi);
    err = fabs((ldexp(yh, -k) - 0.5 * v.hi) - 0.5 * v.lo) / ldexp(0.5, E - 52 - k);
  } else {
    double ys = ldexp(yi, -k);
    err = fabs((ys - v.hi) - v.lo) / ldexp(1.0, E - 52 - k);
  }
  if (same && err > 0.5) err = 0.5;
  st->n_reg++;
  st->sum_ulp += err;
  if (err > st->max_ulp) {
    st->max_ulp = err;
    st->worst = i;
  }
  if (err > bound) {
    st->violations++;
    return 2;
  }
  return 0;
}

/* results y of inputs x against the oracle, the ULP metric of tests/ulp.py
   in binary64 (ulp(v) = 2^(max(floor(log2 |v|), -1022) - 52)); NaN, +-inf,
   +-0 and subnormal correctly rounded results bit for bit (NaN as a class).
   Undecided inputs are listed (their indices) for the ball oracle. */
void oracle_fast64_check(int fn, const double* x, const double* y, long n, double bound,
                         check64_stats* st, long* bad, long bad_cap, long* undec, long undec_cap) {
  memset(st, 0, sizeof(*st));
  st->worst = -1;
  long nb = 0, nu = 0;
  for (long i = 0; i < n; ++i) {
    dd v;
    int k;
    double r, rel;
    int exact = value64(fn, x[i], &v, &k, &r, &rel);
    int c = check_elem(exact, v, k, r, rel, y[i], bound, st, i);
    if (c == 1 && nu < undec_cap) undec[nu++] = i;
    if (c == 2 && nb < bad_cap) bad[nb++] = i;
  }
}

/* the relative error bound the stage claims for each input's pair (0 for
   the exact results) */
void oracle_fast64_rel(int fn, const double* x, long n, double* rel) {
  for (long i = 0; i < n; ++i) {
    dd v;
    int k;
    double r;
    rel[i] = value64(fn, x[i], &v, &k, &r, &rel[i]) ? 0.0 : rel[i];
  }
}

/* ---- pow and atan2 --------------------------------------------------------- */

enum { B_POW, B_ATAN2 };
static const double REL_POW = 0x1p-86, REL_ATAN2 = 0x1p-90;

static int value64_2(int fn, double a, double b, dd* v, int* k, double* rn) {
  if (fn == B_POW) return pow_core(a, b, 710.5, -746.5, v, k, rn);
  return atan2_core(a, b, v, k, rn);
}

void oracle_fast64_eval2(int fn, const double* a, const double* b, long n, double* hi, double* lo,
                         double* rn, uint8_t* undecided) {
  double rel = fn == B_POW ? REL_POW : REL_ATAN2;
  for (long i = 0; i < n; ++i) {
    dd v;
    int k;
    double r;
    if (value64_2(fn, a[i], b[i], &v, &k, &r)) {
      hi[i] = r;
      lo[i] = 0.0;
      rn[i] = r;
      undecided[i] = 0;
      continue;
    }
    undecided[i] = (uint8_t)round_f64(v, k, rel, &r);
    hi[i] = ldexp(v.hi, k);
    lo[i] = ldexp(v.lo, k);
    rn[i] = r;
  }
}

void oracle_fast64_check2(int fn, const double* a, const double* b, const double* y, long n,
                          double bound, check64_stats* st, long* bad, long bad_cap, long* undec,
                          long undec_cap) {
  memset(st, 0, sizeof(*st));
  st->worst = -1;
  double rel = fn == B_POW ? REL_POW : REL_ATAN2;
  long nb = 0, nu = 0;
  for (long i = 0; i < n; ++i) {
    dd v;
    int k;
    double r;
    int exact = value64_2(fn, a[i], b[i], &v, &k, &r);
    int c = check_elem(exact, v, k, r, rel, y[i], bound, st, i);
    if (c == 1 && nu < undec_cap) undec[nu++] = i;
    if (c == 2 && nb < bad_cap) bad[nb++] = i;
  }
}
