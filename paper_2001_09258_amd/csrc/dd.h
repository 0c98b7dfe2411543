// Double-double (T = double) and float-float (T = float) operators.
//
// The paper evaluates 1-ULP functions with simplified double-double
// operators that skip renormalisation unless it is needed (Section 5,
// overview; the operator list is Appendix B's "DD Functions" table).  The
// same set is written here once as a template over the component type, using
// FMA for the exact product error (v_fma_f64 / v_fma_f32 on gfx950):
//
//   dd2_add   (x + y, |x| >= |y| assumed: fast two-sum; paper: ddadd)
//   dd2_add2  (x + y, any order: two-sum;              paper: ddadd2)
//   dd2_mul   (x * y with the exact FMA error term;    paper: ddmul)
//   dd2_squ   (x^2;                                    paper: ddsqu)
//   dd2_div   (x / y;                                  paper: dddiv)
//   dd2_rec   (1 / y)
//   dd2_scale (x * 2^k;                                paper: ddscale)
//   dd2_norm  (renormalise so |lo| <= ulp(hi)/2;       paper: ddnormalize)
//
// Error bounds (relative, u = 2^-53 or 2^-24): two-sum and two-product are
// exact; dd2_add/dd2_add2 of pairs carry ~2u^2 * max(|x|, |y|); dd2_mul ~4u^2;
// dd2_div ~5u^2 once the reciprocal estimate is within ~u of 1/y.
#pragma once
#include "prims.h"
#pragma STDC FP_CONTRACT OFF

namespace lmh {

template <class T>
struct dd2 {
  T hi, lo;
};

template <class T>
LMH_INLINE dd2<T> mk(T hi, T lo) { return dd2<T>{hi, lo}; }

template <class T>
LMH_INLINE T val(dd2<T> a) { return a.hi + a.lo; }

// ---- sums ------------------------------------------------------------------
// |x| >= |y| (or x == 0): s + e == x + y exactly
template <class T>
LMH_INLINE dd2<T> dd2_add(T x, T y) {
  T s = x + y;
  return mk(s, y - (s - x));
}

// any x, y: Knuth's two-sum, s + e == x + y exactly
template <class T>
LMH_INLINE dd2<T> dd2_add2(T x, T y) {
  T s = x + y;
  T v = s - x;
  return mk(s, (x - (s - v)) + (y - v));
}

// pair + scalar, |x| >= |y|
template <class T>
LMH_INLINE dd2<T> dd2_add(dd2<T> x, T y) {
  T s = x.hi + y;
  return mk(s, (y - (s - x.hi)) + x.lo);
}

// scalar + pair, |x| >= |y|
template <class T>
LMH_INLINE dd2<T> dd2_add(T x, dd2<T> y) {
  T s = x + y.hi;
  return mk(s, ((x - s) + y.hi) + y.lo);
}

// pair + pair, |x| >= |y|
template <class T>
LMH_INLINE dd2<T> dd2_add(dd2<T> x, dd2<T> y) {
  T s = x.hi + y.hi;
  return mk(s, (((x.hi - s) + y.hi) + y.lo) + x.lo);
}

// pair + scalar, any order
template <class T>
LMH_INLINE dd2<T> dd2_add2(dd2<T> x, T y) {
  dd2<T> s = dd2_add2(x.hi, y);
  return mk(s.hi, s.lo + x.lo);
}

// pair + pair, any order
template <class T>
LMH_INLINE dd2<T> dd2_add2(dd2<T> x, dd2<T> y) {
  dd2<T> s = dd2_add2(x.hi, y.hi);
  return mk(s.hi, s.lo + (x.lo + y.lo));
}

template <class T>
LMH_INLINE dd2<T> dd2_neg(dd2<T> x) { return mk(-x.hi, -x.lo); }

template <class T>
LMH_INLINE dd2<T> dd2_norm(dd2<T> x) {
  T s = x.hi + x.lo;
  return mk(s, (x.hi - s) + x.lo);
}

template <class T>
LMH_INLINE dd2<T> dd2_scale(dd2<T> x, T s) { return mk(x.hi * s, x.lo * s); }

// ---- products --------------------------------------------------------------
template <class T>
LMH_INLINE dd2<T> dd2_mul(T x, T y) {
  T p = x * y;
  return mk(p, fma_(x, y, -p));
}

template <class T>
LMH_INLINE dd2<T> dd2_mul(dd2<T> x, T y) {
  T p = x.hi * y;
  return mk(p, fma_(x.lo, y, fma_(x.hi, y, -p)));
}

template <class T>
LMH_INLINE dd2<T> dd2_mul(dd2<T> x, dd2<T> y) {
  T p = x.hi * y.hi;
  return mk(p, fma_(x.hi, y.lo, fma_(x.lo, y.hi, fma_(x.hi, y.hi, -p))));
}

template <class T>
LMH_INLINE dd2<T> dd2_squ(dd2<T> x) {
  T p = x.hi * x.hi;
  T t = x.hi + x.hi;
  return mk(p, fma_(t, x.lo, fma_(x.hi, x.hi, -p)));
}

// ---- reciprocal and quotient -----------------------------------------------
// 1/y to about one ulp: hardware estimate plus two Newton steps
template <class T>
LMH_INLINE T rcp_refined(T y) {
  T r = rcp_(y);
  T e = fma_(-y, r, T(1));
  r = fma_(r, e, r);
  e = fma_(-y, r, T(1));
  return fma_(r, e, r);
}

template <class T>
LMH_INLINE dd2<T> dd2_div(dd2<T> n, dd2<T> d) {
  T t = rcp_refined(d.hi);
  T q = n.hi * t;
  T r = fma_(-q, d.hi, n.hi);      // exact residual of the leading part
  r = fma_(-q, d.lo, r) + n.lo;
  T ql = r * t;
  return dd2_add(q, ql);
}

template <class T>
LMH_INLINE dd2<T> dd2_div(T n, dd2<T> d) { return dd2_div(mk(n, T(0)), d); }

template <class T>
LMH_INLINE dd2<T> dd2_rec(dd2<T> d) {
  T t = rcp_refined(d.hi);
  T r = fma_(-t, d.hi, T(1));
  r = fma_(-t, d.lo, r);
  return dd2_add(t, r * t);
}

template <class T>
LMH_INLINE dd2<T> dd2_rec(T d) {
  T t = rcp_refined(d);
  return dd2_add(t, fma_(-t, d, T(1)) * t);
}

// ---- polynomial helpers ----------------------------------------------------
// Horner over a coefficient table, lowest degree first.
template <class T, int N>
LMH_INLINE T poly_horner(T z, const T (&c)[N]) {
  T s = c[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) s = fma_(s, z, c[i]);
  return s;
}

// Estrin's scheme (the paper uses it to shorten FMA dependency chains,
// Section 5, overview): pairs (c0 + c1 z), then combine with z^2, z^4, ...
template <class T, int N>
LMH_INLINE T poly_estrin(T z, const T (&c)[N]) {
  T v[(N + 1) / 2];
#pragma unroll
  for (int i = 0; i < N / 2; ++i) v[i] = fma_(c[2 * i + 1], z, c[2 * i]);
  if (N & 1) v[N / 2] = c[N - 1];
  int m = (N + 1) / 2;
  T zz = z * z;
#pragma unroll
  for (int level = 0; level < 6; ++level) {
    if (m <= 1) break;
#pragma unroll
    for (int i = 0; i < m / 2; ++i) v[i] = fma_(v[2 * i + 1], zz, v[2 * i]);
    if (m & 1) v[m / 2] = v[m - 1];
    m = (m + 1) / 2;
    zz = zz * zz;
  }
  return v[0];
}

// Estrin over the tail c[OFF..N-1] of a table: the polynomial (P(z) - the
// first OFF terms) / z^OFF
template <int OFF, class T, int N>
LMH_INLINE T poly_estrin_tail(T z, const T (&c)[N]) {
  T t[N - OFF];
#pragma unroll
  for (int i = 0; i < N - OFF; ++i) t[i] = c[OFF + i];
  return poly_estrin(z, t);
}

}  // namespace lmh

#pragma STDC FP_CONTRACT DEFAULT
