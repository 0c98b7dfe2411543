/* Double-double arithmetic, the Taylor coefficients and series, and access
 * to the bits of 2/pi, shared by the oracle's fast C stages (fast32.c,
 * fast64.c).  TEST INFRASTRUCTURE ONLY, like the rest of oracle/. */
#pragma once
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "tables.h"

typedef struct {
  double hi, lo;
} dd;

static inline dd two_sum(double a, double b) {
  double s = a + b;
  double v = s - a;
  dd r = {s, (a - (s - v)) + (b - v)};
  return r;
}

static inline dd fast_two_sum(double a, double b) { /* |a| >= |b| or a == 0 */
  double s = a + b;
  dd r = {s, b - (s - a)};
  return r;
}

static inline dd two_prod(double a, double b) {
  double p = a * b;
  dd r = {p, fma(a, b, -p)};
  return r;
}

static inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

static inline dd dd_neg(dd a) {
  dd r = {-a.hi, -a.lo};
  return r;
}

static inline dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}

static inline dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return fast_two_sum(p.hi, p.lo);
}

static inline dd dd_div(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd r = dd_add(a, dd_neg(dd_mul_d(b, q1)));
  double q2 = r.hi / b.hi;
  r = dd_add(r, dd_neg(dd_mul_d(b, q2)));
  double q3 = r.hi / b.hi;
  dd q = fast_two_sum(q1, q2);
  return dd_add(q, (dd){q3, 0.0});
}

static inline dd dd_from(double a) {
  dd r = {a, 0.0};
  return r;
}

/* ---- the series ------------------------------------------------------- */

/* Taylor coefficients as pairs, formed once when the library is loaded:
   1/n! by repeated pair division, 1/(2k + 1) likewise (each within 2^-104) */
#define NFACT 32
#define NODD 24
static dd INV_FACT[NFACT];
static dd INV_ODD[NODD];

static dd INV_LN2;

__attribute__((constructor)) static void init_coefficients(void) {
  INV_LN2 = dd_div(dd_from(1.0), (dd){LN2_D[0], LN2_D[1]});
  INV_FACT[0] = dd_from(1.0);
  for (int n = 1; n < NFACT; ++n) INV_FACT[n] = dd_div(INV_FACT[n - 1], dd_from((double)n));
  for (int k = 0; k < NODD; ++k) INV_ODD[k] = dd_div(dd_from(1.0), dd_from((double)(2 * k + 1)));
}

/* Horner's rule for a polynomial in z whose coefficients from index LO up
   contribute less than 2^-57 of the sum: those in binary64, the rest in
   pairs.  One polynomial evaluation, coefficient k of c at c[k * stride +
   off]. */
static dd horner(dd z, const dd* c, int stride, int off, int top, int lo) {
  double t = c[top * stride + off].hi;
  for (int k = top - 1; k >= lo; --k) t = t * z.hi + c[k * stride + off].hi;
  dd s = dd_from(t);
  for (int k = lo - 1; k >= 0; --k) s = dd_add(dd_mul(s, z), c[k * stride + off]);
  return s;
}

/* sin r = r sum_{n<=13} (-r^2)^n / (2n+1)!  and cos r = sum_{n<=14} (-r^2)^n
   / (2n)! for |r| <= pi/4 (+ 2^-40): the first omitted terms are below
   2^-112 |sin r| and 2^-117; the terms from n = 9 on are below 2^-63 and
   summed in binary64 */
static dd sin_series(dd r) {
  dd z = dd_neg(dd_mul(r, r));
  return dd_mul(horner(z, INV_FACT, 2, 1, 13, 9), r);
}

static dd cos_series(dd r) {
  dd z = dd_neg(dd_mul(r, r));
  return horner(z, INV_FACT, 2, 0, 14, 10);
}

/* e^r = sum_{n<=23} r^n / n! for |r| <= 0.35: the first omitted term is
   below 2^-115; the terms from n = 14 on are below 2^-57 */
static dd exp_series(dd r) { return horner(r, INV_FACT, 1, 0, 23, 14); }

/* 2 atanh t = 2 t sum_{k<=21} t^(2k) / (2k+1) for |t| <= 0.172: the first
   omitted term is below 2^-112 of the sum; the terms from k = 12 on are
   below 2^-60 */
static dd atanh2_series(dd t) {
  dd s = dd_mul(horner(dd_mul(t, t), INV_ODD, 1, 0, 21, 12), t);
  s.hi *= 2.0;
  s.lo *= 2.0;
  return s;
}

/* ---- reductions --------------------------------------------------------- */

/* 32 bits of 2/pi's fraction starting at bit position p (0-based: bit 0
   has weight 1/2); bits past the table are zero */
static uint32_t tbits32(int p) {
  int w = p / 32, o = p % 32;
  uint32_t a = w < TWO_OVER_PI_WORDS ? TWO_OVER_PI_W[w] : 0u;
  uint32_t b = w + 1 < TWO_OVER_PI_WORDS ? TWO_OVER_PI_W[w + 1] : 0u;
  return o ? (a << o) | (b >> (32 - o)) : a;
}

/* bits [lowbit, lowbit + 63] of the little-endian number Q of nq 64-bit words */
static uint64_t get64n(const uint64_t* Q, int nq, int lowbit) {
  if (lowbit < 0) return get64n(Q, nq, 0) << -lowbit;
  int w = lowbit / 64, o = lowbit % 64;
  uint64_t a = w < nq ? Q[w] : 0u;
  uint64_t b = w + 1 < nq ? Q[w + 1] : 0u;
  return o ? (a >> o) | (b << (64 - o)) : a;
}


/* e^a as a pair (finite |a| <= 708: the result stays a normal double) */
static dd exp_pair(double a) {
  double k = nearbyint(a / LN2_D[0]);
  dd r = dd_add(dd_from(a), dd_neg(two_prod(k, LN2_D[0])));
  r = dd_add(r, dd_neg(two_prod(k, LN2_D[1])));
  r = dd_add(r, dd_from(-k * LN2_D[2]));
  dd e = exp_series(r);
  e.hi = ldexp(e.hi, (int)k);
  e.lo = ldexp(e.lo, (int)k);
  return e;
}

/* sinh, cosh, tanh from E = e^|x| as a pair; below |x| = 2^-4 sinh and tanh
   by their Taylor series (x + x^3/6 + ... and x - x^3/3 + ...), where E - 1/E
   would cancel */
static dd sinh_small(dd x) { /* |x| < 2^-4: sum x^(2n+1)/(2n+1)!, n <= 8 */
  dd z = dd_mul(x, x);
  dd s = INV_FACT[17];
  for (int n = 7; n >= 0; --n) s = dd_add(dd_mul(s, z), INV_FACT[2 * n + 1]);
  return dd_mul(s, x);
}

