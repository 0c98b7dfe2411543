/*
 * libm_hip -- elementwise C99 real math functions on AMD Instinct MI355X
 * (gfx950), after N. Shibata and F. Petrogalli, "SLEEF: A Portable
 * Vectorized Library of C Standard Mathematical Functions" (IEEE TPDS 2020).
 *
 * One entry point per (function, accuracy variant, element type) over device
 * arrays.  Semantics follow the paper's library contract (Section 5,
 * "Overview of Library Implementation" and "Handling of Special Numbers"):
 *
 *   - u10 variants are within 1.0 ULP of the exact result, u35 variants
 *     within 3.5 ULP; fmod and remainder are exact;
 *   - special arguments (zeros, infinities, NaN) give the values C99 Annex F
 *     prescribes; no errno, no floating-point exception flags;
 *   - round-to-nearest mode only; subnormal inputs and outputs are honoured.
 *
 * Conventions shared by every entry point
 *   pointers   device pointers (hipMalloc / torch allocations on the current
 *              device).  Any alignment is accepted; 16-byte aligned arrays use
 *              128-bit loads and stores.  The caller owns all buffers.
 *   n          element count (64-bit); n == 0 returns LIBM_HIP_OK and launches
 *              nothing.
 *   aliasing   in place (out == an input) is allowed; partial overlap is not.
 *   stream     a hipStream_t passed as void* (NULL = the null stream).  Calls
 *              only enqueue work: they return before the results exist.
 *   errors     LIBM_HIP_ERR_INVALID for a NULL pointer with n > 0 (checked
 *              before any HIP call), LIBM_HIP_ERR_UNSUPPORTED for an unknown
 *              combination in the generic dispatcher, LIBM_HIP_ERR_HIP when
 *              the kernel launch fails; libm_hip_last_error() then returns a
 *              thread-local message.  There are no per-element errors.
 *   threads    every call is thread-safe.
 *
 * Element types: f64 = double, f32 = float, bf16 and f16 = uint16_t bit
 * patterns of bfloat16 / IEEE binary16 (evaluated in binary32 and rounded to
 * nearest-even once).  "f32_via_f64" variants take and return float but
 * evaluate in binary64 and round once.  bf16 and f16 run evaluators sized
 * for those formats where they exist (exp, exp2, log, log2, pow, sinh, cosh,
 * tanh; sin, cos, tan and sincos: binary32 arithmetic with short series and
 * the transcendental unit, every one of the 65536 inputs of each format
 * within 1.0 ULP); otherwise these forms run the wider type's 3.5-ULP
 * evaluator where the function has one (asin, acos, atan, atan2, and for
 * f32_via_f64 also sin, cos, tan, sincos, log, sinh, cosh, tanh), else its
 * 1.0-ULP one: the wider type carries at least 13 more bits, so the result
 * is within 0.5 + 3.5 * 2^-13 ULP of the exact value in the narrow format.
 */
#ifndef LIBM_HIP_H
#define LIBM_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LIBM_HIP_OK = 0,
  LIBM_HIP_ERR_INVALID = 1,
  LIBM_HIP_ERR_UNSUPPORTED = 2,
  LIBM_HIP_ERR_HIP = 3,
  LIBM_HIP_ERR_NOMEM = 4
} libm_hip_status;

/* Message describing the last error on the calling thread ("" if none). */
const char* libm_hip_last_error(void);
/* Library version string. */
const char* libm_hip_version(void);

/* ------------------------------------------------------------------------
 * Unary functions, y[i] = f(x[i]).
 *
 * sin, cos, tan (Section 5, "sin and cos", "tan", "The Payne-Hanek Range
 * Reduction"): a Cody-Waite reduction for |x| < 2^14 (binary32: 65536) and
 * the vectorised Payne-Hanek reduction above, chosen per element (the
 * paper's bit-consistent arrangement, Section 3.3); a sine polynomial on
 * [-pi/2, pi/2]; tan through the double-angle formula on [-pi/8, pi/8].
 * exp (Section 5, "exp"), log (Section 5, "log"; also a 3.5-ULP form).  asin, acos (Section 5,
 * "asin and acos": reduction to [0, 0.5] through sqrt((1-x)/2)) and atan
 * (Section 5, "atan": reduction to [0, 1] through 1/x).  exp2, log2, sinh,
 * cosh and tanh are not described in the paper and are built from the same
 * reductions and double-double pieces; their 3.5-ULP forms (binary64 and
 * binary32) drop the double-double: e^|x|/2 in working precision and one
 * IEEE division.  log10, log1p, exp10, expm1 and cbrt
 * belong to the C99 set the paper's library provides (Section 1) but are
 * not described either: log10 and log1p through the log reduction (log1p
 * with 1 + x kept as an exact pair), exp10 and expm1 through the exp
 * reduction (expm1 with e^r - 1 as a pair and 2^k - 1 as an exact pair),
 * cbrt by Newton steps on x^(-1/3) from the hardware log2/exp2 estimates and
 * one double-double residual correction.  asinh, acosh and atanh (C99, not
 * described in the paper either) as log1p of an argument formed without
 * cancellation: |x| + x^2/(1 + sqrt(1 + x^2)), (x - 1) + sqrt((x - 1)(x + 1))
 * and 2|x|/(1 - |x|) (halved), in double-double (binary32: in binary64
 * working precision).  erf and erfc (C99, not described in the paper):
 * erf x = c0 x + c1 x^3 + x^5 P(x^2) below |x| = 0.75 (c0, c1 as pairs);
 * above, erfc |x| = e^(-x^2) g(|x|) with g from a six-row table of
 * polynomials (in |x|, or in 1/|x| from 2.25 on) and e^(-x^2) from the
 * double-double exp of the exact square; erf = 1 - erfc there, erfc(-|x|) =
 * 2 - erfc |x| (binary32: the same in binary64 working precision).  All 1.0
 * ULP; the same Annex F special values as C99 (exp10 as exp: 10^+-0 = 1,
 * 10^-inf = +0; erf(+-0) = +-0, erf(+-inf) = +-1, erfc(-inf) = 2,
 * erfc(+inf) = +0).
 * ---------------------------------------------------------------------- */
#define LIBM_HIP_DECL_UNARY(fn, var)                                                       \
  libm_hip_status libm_hip_##fn##_##var##_f64(const double* x, double* y, size_t n,        \
                                              void* stream);                               \
  libm_hip_status libm_hip_##fn##_##var##_f32(const float* x, float* y, size_t n,          \
                                              void* stream);
#define LIBM_HIP_DECL_UNARY_HALF(fn)                                                       \
  libm_hip_status libm_hip_##fn##_u10_bf16(const uint16_t* x, uint16_t* y, size_t n,       \
                                           void* stream);                                  \
  libm_hip_status libm_hip_##fn##_u10_f16(const uint16_t* x, uint16_t* y, size_t n,        \
                                          void* stream);                                   \
  libm_hip_status libm_hip_##fn##_u10_f32_via_f64(const float* x, float* y, size_t n,      \
                                                  void* stream);

LIBM_HIP_DECL_UNARY(sin, u10)
LIBM_HIP_DECL_UNARY(sin, u35)
LIBM_HIP_DECL_UNARY(cos, u10)
LIBM_HIP_DECL_UNARY(cos, u35)
LIBM_HIP_DECL_UNARY(tan, u10)
LIBM_HIP_DECL_UNARY(tan, u35)
LIBM_HIP_DECL_UNARY(exp, u10)
LIBM_HIP_DECL_UNARY(exp2, u10)
LIBM_HIP_DECL_UNARY(log, u10)
LIBM_HIP_DECL_UNARY(log, u35)
LIBM_HIP_DECL_UNARY(log2, u10)
LIBM_HIP_DECL_UNARY(sinh, u10)
LIBM_HIP_DECL_UNARY(cosh, u10)
LIBM_HIP_DECL_UNARY(tanh, u10)
LIBM_HIP_DECL_UNARY(sinh, u35)
LIBM_HIP_DECL_UNARY(cosh, u35)
LIBM_HIP_DECL_UNARY(tanh, u35)
LIBM_HIP_DECL_UNARY(asin, u10)
LIBM_HIP_DECL_UNARY(asin, u35)
LIBM_HIP_DECL_UNARY(acos, u10)
LIBM_HIP_DECL_UNARY(acos, u35)
LIBM_HIP_DECL_UNARY(atan, u10)
LIBM_HIP_DECL_UNARY(atan, u35)
LIBM_HIP_DECL_UNARY_HALF(sin)
LIBM_HIP_DECL_UNARY_HALF(cos)
LIBM_HIP_DECL_UNARY_HALF(tan)
LIBM_HIP_DECL_UNARY_HALF(exp)
LIBM_HIP_DECL_UNARY_HALF(exp2)
LIBM_HIP_DECL_UNARY_HALF(log)
LIBM_HIP_DECL_UNARY_HALF(log2)
LIBM_HIP_DECL_UNARY_HALF(sinh)
LIBM_HIP_DECL_UNARY_HALF(cosh)
LIBM_HIP_DECL_UNARY_HALF(tanh)
LIBM_HIP_DECL_UNARY_HALF(asin)
LIBM_HIP_DECL_UNARY_HALF(acos)
LIBM_HIP_DECL_UNARY_HALF(atan)
LIBM_HIP_DECL_UNARY(log10, u10)
LIBM_HIP_DECL_UNARY(log1p, u10)
LIBM_HIP_DECL_UNARY(exp10, u10)
LIBM_HIP_DECL_UNARY(expm1, u10)
LIBM_HIP_DECL_UNARY(cbrt, u10)
LIBM_HIP_DECL_UNARY_HALF(log10)
LIBM_HIP_DECL_UNARY_HALF(log1p)
LIBM_HIP_DECL_UNARY_HALF(exp10)
LIBM_HIP_DECL_UNARY_HALF(expm1)
LIBM_HIP_DECL_UNARY_HALF(cbrt)
LIBM_HIP_DECL_UNARY(asinh, u10)
LIBM_HIP_DECL_UNARY(acosh, u10)
LIBM_HIP_DECL_UNARY(atanh, u10)
LIBM_HIP_DECL_UNARY(erf, u10)
LIBM_HIP_DECL_UNARY(erfc, u10)
LIBM_HIP_DECL_UNARY_HALF(asinh)
LIBM_HIP_DECL_UNARY_HALF(acosh)
LIBM_HIP_DECL_UNARY_HALF(atanh)
LIBM_HIP_DECL_UNARY_HALF(erf)
LIBM_HIP_DECL_UNARY_HALF(erfc)

/* lgamma and tgamma (C99 functions of the paper's set, Section 1; not
 * described in the paper).  log Gamma(a) for a > 0 as a double-double pair:
 * minimax expansions around the zeros at 1 and 2 (|a - 1|, |a - 2| <= 1/16),
 * Stirling's series with ten Bernoulli terms from a >= 10, and below that
 * the recurrence up to a + n >= 10 with the product a (a + 1) ... (a + n - 1)
 * in double-double; lgamma(x) = log Gamma(1 + x) - log|x| for |x| < 1/16 and
 * the reflection formula for x <= -1/16; tgamma = sign e^lgamma, the
 * exponential of the pair rounded once.  1.0 ULP, except next to the zeros
 * of lgamma on the negative axis (where the reflection's subtraction
 * cancels; the error there is about 2^-100 absolute).  binary32: the binary64
 * pairs rounded once.  Annex F: lgamma(+-0) = lgamma(-n) = lgamma(+-inf) =
 * +inf, lgamma(1) = lgamma(2) = +0; tgamma(+-0) = +-inf, tgamma(-n) =
 * tgamma(-inf) = NaN, tgamma(+inf) = +inf; NaN gives NaN. */
LIBM_HIP_DECL_UNARY(lgamma, u10)
LIBM_HIP_DECL_UNARY(tgamma, u10)
LIBM_HIP_DECL_UNARY_HALF(lgamma)
LIBM_HIP_DECL_UNARY_HALF(tgamma)

/* ------------------------------------------------------------------------
 * sincos: s[i] = sin(x[i]) and c[i] = cos(x[i]) in one pass (the paper's
 * library provides sincos, Section 1).  Each result is bit-identical to the
 * sin and cos entry points of the same variant and type: the Cody-Waite
 * elements take sin's and cos's own reductions, a Payne-Hanek element is
 * reduced once and mapped to both.  u10: f64, f32, bf16, f16, f32_via_f64;
 * u35: f64, f32.  s and c are distinct outputs; either may be x itself
 * (in-place); NULL x, s or c with n > 0 -> LIBM_HIP_ERR_INVALID.
 * ---------------------------------------------------------------------- */
#define LIBM_HIP_DECL_SINCOS(var, T, tag)                                                  \
  libm_hip_status libm_hip_sincos_##var##_##tag(const T* x, T* s, T* c, size_t n,          \
                                                void* stream);
LIBM_HIP_DECL_SINCOS(u10, double, f64)
LIBM_HIP_DECL_SINCOS(u10, float, f32)
LIBM_HIP_DECL_SINCOS(u10, uint16_t, bf16)
LIBM_HIP_DECL_SINCOS(u10, uint16_t, f16)
LIBM_HIP_DECL_SINCOS(u10, float, f32_via_f64)
LIBM_HIP_DECL_SINCOS(u35, double, f64)
LIBM_HIP_DECL_SINCOS(u35, float, f32)

/* ------------------------------------------------------------------------
 * Binary functions, C argument order.
 *
 * pow(x, y) (Section 5, "pow": e^(y log x) in double-double), out = x^y.
 * atan2(y, x): quadrant logic around the atan polynomial on [0, 1]
 *   (Section 5, "atan"); out = atan2(y, x).  The 3.5-ULP form (binary64 and
 *   binary32) takes the ratio by one IEEE division and evaluates the
 *   polynomial and the pi/2, pi reconstructions in working precision.
 * hypot(x, y): sqrt(x^2 + y^2) without intermediate overflow or underflow
 *   (C99; not described in the paper): the larger magnitude scaled into
 *   [0.5, 1), the sum of squares as a double-double pair, a reciprocal
 *   square root estimate refined by Newton steps and one residual
 *   correction; 1.0 ULP; an infinite argument gives +inf even with a NaN.
 * fmod(x, y), remainder(x, y): exact; long division with floating-point
 *   digits (Section 5, "FP Remainder", Algorithm 1, Appendices B and C),
 *   extended to quotients beyond DBL_MAX.  remainder rounds the quotient to
 *   nearest-even (IEEE 754).
 * fdim(x, y), fmax(x, y), fmin(x, y): exact (C99 F.9.9; the paper shows
 *   fdim as a masking example, Section 2): fdim is x - y rounded once when
 *   x > y, else +0, NaN if either argument is NaN; fmax / fmin return the
 *   larger / smaller argument, the other one when one is NaN, NaN when both
 *   are; -0 counts as smaller than +0 (C99 leaves that order open).
 * copysign(x, y), nextafter(x, y): exact (C99 F.9.8.3, F.9.8.3's neighbour
 *   rule: y if x == y, the smallest subnormal towards y from a zero, NaN if
 *   either argument is NaN).
 * ---------------------------------------------------------------------- */
#define LIBM_HIP_DECL_BINARY(fn, var, T, tag)                                              \
  libm_hip_status libm_hip_##fn##var##_##tag(const T* a, const T* b, T* out, size_t n,     \
                                             void* stream);
LIBM_HIP_DECL_BINARY(pow, _u10, double, f64)
LIBM_HIP_DECL_BINARY(pow, _u10, float, f32)
LIBM_HIP_DECL_BINARY(pow, _u10, uint16_t, bf16)
LIBM_HIP_DECL_BINARY(pow, _u10, uint16_t, f16)
LIBM_HIP_DECL_BINARY(pow, _u10, float, f32_via_f64)
LIBM_HIP_DECL_BINARY(atan2, _u10, double, f64)
LIBM_HIP_DECL_BINARY(atan2, _u10, float, f32)
LIBM_HIP_DECL_BINARY(atan2, _u10, uint16_t, bf16)
LIBM_HIP_DECL_BINARY(atan2, _u10, uint16_t, f16)
LIBM_HIP_DECL_BINARY(atan2, _u10, float, f32_via_f64)
LIBM_HIP_DECL_BINARY(atan2, _u35, double, f64)
LIBM_HIP_DECL_BINARY(atan2, _u35, float, f32)
LIBM_HIP_DECL_BINARY(pow, _u35, double, f64)
LIBM_HIP_DECL_BINARY(pow, _u35, float, f32)
LIBM_HIP_DECL_BINARY(hypot, _u10, double, f64)
LIBM_HIP_DECL_BINARY(hypot, _u10, float, f32)
LIBM_HIP_DECL_BINARY(hypot, _u10, uint16_t, bf16)
LIBM_HIP_DECL_BINARY(hypot, _u10, uint16_t, f16)
LIBM_HIP_DECL_BINARY(hypot, _u10, float, f32_via_f64)
LIBM_HIP_DECL_BINARY(fmod, , double, f64)
LIBM_HIP_DECL_BINARY(fmod, , float, f32)
LIBM_HIP_DECL_BINARY(remainder, , double, f64)
LIBM_HIP_DECL_BINARY(remainder, , float, f32)
LIBM_HIP_DECL_BINARY(fdim, , double, f64)
LIBM_HIP_DECL_BINARY(fdim, , float, f32)
LIBM_HIP_DECL_BINARY(fmax, , double, f64)
LIBM_HIP_DECL_BINARY(fmax, , float, f32)
LIBM_HIP_DECL_BINARY(fmin, , double, f64)
LIBM_HIP_DECL_BINARY(fmin, , float, f32)
LIBM_HIP_DECL_BINARY(copysign, , double, f64)
LIBM_HIP_DECL_BINARY(copysign, , float, f32)
LIBM_HIP_DECL_BINARY(nextafter, , double, f64)
LIBM_HIP_DECL_BINARY(nextafter, , float, f32)

/* ------------------------------------------------------------------------
 * The rest of the C99 real functions with one exact answer (the paper's
 * library covers all C99 real functions, Section 1), binary64 and binary32,
 * y[i] = f(x[i]): sqrt correctly rounded (the IEEE square root), trunc,
 * floor, ceil, round (halfway cases away from zero), rint (halfway cases to
 * even), fabs, logb (the exponent of x as if normalized; logb(+-0) = -inf,
 * logb(+-inf) = +inf).  Signs of zero and NaN as C99 Annex F.
 * ---------------------------------------------------------------------- */
#define LIBM_HIP_DECL_EXACT1(fn)                                                            \
  libm_hip_status libm_hip_##fn##_f64(const double* x, double* y, size_t n, void* stream);  \
  libm_hip_status libm_hip_##fn##_f32(const float* x, float* y, size_t n, void* stream);
LIBM_HIP_DECL_EXACT1(sqrt)
LIBM_HIP_DECL_EXACT1(trunc)
LIBM_HIP_DECL_EXACT1(floor)
LIBM_HIP_DECL_EXACT1(ceil)
LIBM_HIP_DECL_EXACT1(round)
LIBM_HIP_DECL_EXACT1(rint)
LIBM_HIP_DECL_EXACT1(fabs)
LIBM_HIP_DECL_EXACT1(logb)

/* ------------------------------------------------------------------------
 * C99 functions with integer operands or results (7.12.6; the paper's
 * library covers all C99 real functions, Section 1), binary64 and binary32,
 * one element per index, integer arrays of int32_t:
 *   ldexp:  y[i] = x[i] * 2^e[i] rounded once (scalbn is the same function
 *           for binary formats); exponents beyond +-2200 (binary32: +-400)
 *           act as those bounds, where every finite nonzero x already
 *           overflows or underflows.
 *   ilogb:  e[i] = the exponent of x[i] as if normalized; INT_MIN for +-0
 *           and NaN (FP_ILOGB0 = FP_ILOGBNAN), INT_MAX for +-inf.
 *   frexp:  m[i] in [0.5, 1) with x[i] = m[i] * 2^e[i]; +-0, +-inf and NaN
 *           give m[i] = x[i], e[i] = 0.
 *   modf:   f[i] = x[i] - trunc(x[i]), ip[i] = trunc(x[i]), both with the
 *           sign of x[i]; +-inf gives (+-0, +-inf), NaN (NaN, NaN).
 *   fma:    y[i] = a[i] * b[i] + c[i] rounded once (IEEE fused multiply-add).
 *   remquo: r[i] = remainder(x[i], y[i]) (bit-identical to the remainder
 *           entry point), q[i] with the sign of x/y and the low three bits
 *           of the magnitude of the quotient rounded to nearest-even; q = 0
 *           where the remainder is NaN or y is infinite.
 *   lrint, lround: the nearest integer of x[i] as int64_t (halfway cases to
 *           even / away from zero); INT64_MIN where it does not fit in
 *           int64_t and for NaN (C99 leaves those unspecified).
 * Exact.  Any alignment; not served by libm_hip_eval or the batch API
 * (their requests carry one or two floating-point operands and one result).
 * ---------------------------------------------------------------------- */
#define LIBM_HIP_DECL_MAPS(T, tag)                                                           \
  libm_hip_status libm_hip_modf_##tag(const T* x, T* f, T* ip, size_t n, void* stream);    \
  libm_hip_status libm_hip_fma_##tag(const T* a, const T* b, const T* c, T* y, size_t n,   \
                                     void* stream);                                         \
  libm_hip_status libm_hip_lrint_##tag(const T* x, int64_t* y, size_t n, void* stream);    \
  libm_hip_status libm_hip_lround_##tag(const T* x, int64_t* y, size_t n, void* stream);   \
  libm_hip_status libm_hip_remquo_##tag(const T* x, const T* y, T* r, int32_t* q, size_t n, \
                                        void* stream);
LIBM_HIP_DECL_MAPS(double, f64)
LIBM_HIP_DECL_MAPS(float, f32)
libm_hip_status libm_hip_ldexp_f64(const double* x, const int32_t* e, double* y, size_t n,
                                   void* stream);
libm_hip_status libm_hip_ldexp_f32(const float* x, const int32_t* e, float* y, size_t n,
                                   void* stream);
libm_hip_status libm_hip_ilogb_f64(const double* x, int32_t* e, size_t n, void* stream);
libm_hip_status libm_hip_ilogb_f32(const float* x, int32_t* e, size_t n, void* stream);
libm_hip_status libm_hip_frexp_f64(const double* x, double* m, int32_t* e, size_t n,
                                   void* stream);
libm_hip_status libm_hip_frexp_f32(const float* x, float* m, int32_t* e, size_t n,
                                   void* stream);

/* ------------------------------------------------------------------------
 * Backward (vector-Jacobian products) for autograd; not part of the paper.
 * gx[i] = gy[i] * f'(x[i]) for sin, cos, tan, exp, log, tanh, evaluated from
 * the u10 forward pieces (tanh' as 1/cosh^2, never 1 - tanh^2).  Binary:
 *   pow:   gx = gout * y * x^(y-1),  gy = gout * x^y * log(x)  (x > 0, and
 *          x < 0 with integer y for gx; each rounded once, also where the
 *          power or the product over- or underflows); at x == +-0 gx =
 *          gout * y * pow(x, y - 1) with Annex F pow (0 for y == 0) and gy
 *          = 0 for y >= 0, NaN for y < 0; gy is NaN for x < 0, both are NaN
 *          for x < 0 with non-integer y;
 *   atan2: gy = gout * x / (x^2 + y^2), gx = -gout * y / (x^2 + y^2), with x
 *          and y scaled by a common power of two (no overflow or underflow
 *          of the squares); both NaN at (0, 0).
 * Bounds (against the correctly rounded products): 2.5 ULP for the unary
 * gradients, 4 ULP for the pow and atan2 partials.
 * Same conventions as the forward calls (device pointers, n, stream).
 * ---------------------------------------------------------------------- */
#define LIBM_HIP_DECL_BWD(fn)                                                              \
  libm_hip_status libm_hip_##fn##_u10_f64_bwd(const double* x, const double* gy,           \
                                              double* gx, size_t n, void* stream);         \
  libm_hip_status libm_hip_##fn##_u10_f32_bwd(const float* x, const float* gy, float* gx,  \
                                              size_t n, void* stream);
LIBM_HIP_DECL_BWD(sin)
LIBM_HIP_DECL_BWD(cos)
LIBM_HIP_DECL_BWD(tan)
LIBM_HIP_DECL_BWD(exp)
LIBM_HIP_DECL_BWD(log)
LIBM_HIP_DECL_BWD(tanh)
libm_hip_status libm_hip_pow_u10_f64_bwd(const double* x, const double* y, const double* gout,
                                         double* gx, double* gy, size_t n, void* stream);
libm_hip_status libm_hip_pow_u10_f32_bwd(const float* x, const float* y, const float* gout,
                                         float* gx, float* gy, size_t n, void* stream);
libm_hip_status libm_hip_atan2_u10_f64_bwd(const double* y, const double* x, const double* gout,
                                           double* gy, double* gx, size_t n, void* stream);
libm_hip_status libm_hip_atan2_u10_f32_bwd(const float* y, const float* x, const float* gout,
                                           float* gy, float* gx, size_t n, void* stream);

/* ------------------------------------------------------------------------
 * Generic dispatcher: the same kernels selected by enums.  b must be NULL
 * for unary functions.  Returns LIBM_HIP_ERR_UNSUPPORTED for a combination
 * the library does not serve (e.g. u35 in bf16).
 * ---------------------------------------------------------------------- */
typedef enum {
  LIBM_HIP_SIN = 0, LIBM_HIP_COS, LIBM_HIP_TAN, LIBM_HIP_EXP, LIBM_HIP_EXP2,
  LIBM_HIP_LOG, LIBM_HIP_LOG2, LIBM_HIP_POW, LIBM_HIP_ATAN2, LIBM_HIP_SINH,
  LIBM_HIP_COSH, LIBM_HIP_TANH, LIBM_HIP_FMOD, LIBM_HIP_REMAINDER,
  LIBM_HIP_ASIN, LIBM_HIP_ACOS, LIBM_HIP_ATAN,
  LIBM_HIP_LOG10, LIBM_HIP_LOG1P, LIBM_HIP_EXP10, LIBM_HIP_EXPM1, LIBM_HIP_CBRT,
  LIBM_HIP_HYPOT, LIBM_HIP_ASINH, LIBM_HIP_ACOSH, LIBM_HIP_ATANH,
  LIBM_HIP_ERF, LIBM_HIP_ERFC, LIBM_HIP_FDIM, LIBM_HIP_FMAX, LIBM_HIP_FMIN,
  LIBM_HIP_SQRT, LIBM_HIP_TRUNC, LIBM_HIP_FLOOR, LIBM_HIP_CEIL, LIBM_HIP_ROUND, LIBM_HIP_RINT,
  LIBM_HIP_FABS, LIBM_HIP_LOGB, LIBM_HIP_COPYSIGN, LIBM_HIP_NEXTAFTER,
  LIBM_HIP_LGAMMA, LIBM_HIP_TGAMMA,
  LIBM_HIP_NUM_FN
} libm_hip_fn;
typedef enum { LIBM_HIP_U10 = 0, LIBM_HIP_U35 = 1, LIBM_HIP_EXACT = 2 } libm_hip_variant;
typedef enum {
  LIBM_HIP_F64 = 0, LIBM_HIP_F32 = 1, LIBM_HIP_BF16 = 2, LIBM_HIP_F16 = 3,
  LIBM_HIP_F32_VIA_F64 = 4
} libm_hip_dtype;

libm_hip_status libm_hip_eval(libm_hip_fn fn, libm_hip_variant v, libm_hip_dtype t,
                              const void* a, const void* b, void* out, size_t n,
                              void* stream);

/* ------------------------------------------------------------------------
 * Bit-consistent form (the paper's bit-wise consistent functions, Section
 * 3.3): the same evaluators with every primitive an IEEE operation with a
 * defined result (correctly rounded division and square root in place of
 * the hardware reciprocal, reciprocal square root and log2/exp2 estimates;
 * a seed for x^(-1/3) from fused multiply-adds only) and every element on
 * its own path.  Its results equal, bit for bit, those of the host build of
 * the same source, libm_hip_host_eval (libm_hip_host.h), so a CPU can
 * reproduce them.  Arguments and status as for libm_hip_eval, with t
 * LIBM_HIP_F64 or LIBM_HIP_F32 only (others: LIBM_HIP_ERR_UNSUPPORTED);
 * every (fn, v) of the library is served.  Same accuracy bounds and special
 * values as the default entry points, which may differ from it in the last
 * bit of some results; one plain kernel (an element per lane), slower than
 * the default entry points.
 * ---------------------------------------------------------------------- */
libm_hip_status libm_hip_consistent_eval(libm_hip_fn fn, libm_hip_variant v, libm_hip_dtype t,
                                         const void* a, const void* b, void* out, size_t n,
                                         void* stream);

/* ------------------------------------------------------------------------
 * Launch-shape autotuner (not part of the paper).  Every entry point except
 * the trigonometric ones (whose kernel gathers Payne-Hanek lanes through a
 * queue sized to a 256-lane workgroup) launches with a (workgroup size,
 * 16-byte packs per lane) pair looked up per entry point and size bucket
 * floor(log2 n); the default is (256, 1).
 *
 * libm_hip_tune: times every pair in {64, 128, 256, 512, 1024} x {1, 2, 4}
 *   on the caller's buffers (one warm-up and the fastest of three rounds of
 *   three launches each, HIP events on `stream`; it waits for the stream),
 *   records the fastest for (fn, v, t, bucket of n) if it beats the default
 *   (256, 1) by at least 2% (else the default) and returns it.  The buffers
 *   are overwritten with valid results.  sin, cos and tan have the fixed
 *   shape (256, 1): the call returns it without launching anything.
 * libm_hip_tune_save / _load: the table as text lines "key bucket block packs";
 *   the environment variable LIBM_HIP_TUNE_CACHE names a file loaded at the
 *   first launch.  libm_hip_tune_reset restores the defaults.
 * ---------------------------------------------------------------------- */
libm_hip_status libm_hip_tune(libm_hip_fn fn, libm_hip_variant v, libm_hip_dtype t,
                              const void* a, const void* b, void* out, size_t n, void* stream,
                              int* best_block, int* best_packs);
libm_hip_status libm_hip_tune_save(const char* path);
libm_hip_status libm_hip_tune_load(const char* path);
void libm_hip_tune_reset(void);

/* ------------------------------------------------------------------------
 * Batched evaluation (not part of the paper): one persistent kernel, captured
 * once in a hip graph per plan, serves a list of requests of uneven lengths.
 * Results are bit-identical to the per-function entry points (same
 * evaluators).  Requests are cut into 4096-element tiles that workgroups take
 * from a device counter, most expensive requests first.
 *
 * libm_hip_batch_plan_create: makes a plan on `device` (-1: the calling
 *   thread's current device), allocating there the device request table (up
 *   to max_requests <= 1024 entries), a tile counter, a pinned staging copy
 *   and a private capture stream.  The plan owns these; destroy frees them
 *   (call it once the plan's last run has completed, e.g. after synchronizing
 *   its stream).  The persistent grid holds as many 256-lane workgroups per
 *   CU as can be resident together.  Runs replay a captured hip graph.
 * libm_hip_batch_plan_set_graph: use_graph = 0 makes later runs launch the
 *   kernels directly instead of replaying the graph (same results).
 * libm_hip_batch_run: validates every request (LIBM_HIP_ERR_UNSUPPORTED for a
 *   combination the library does not serve, LIBM_HIP_ERR_INVALID for NULL
 *   pointers with n > 0), uploads the table on `stream` (a stream of the
 *   plan's device) and enqueues the kernels there; returns without waiting
 *   for them.  Requests with n == 0 are skipped.  A plan is not thread-safe:
 *   runs of one plan must be issued from one thread, on one stream or with
 *   the streams ordered by the caller.
 * Errors of these calls are reported by libm_hip_last_error() (the calling
 * thread's message); libm_hip_batch_last_error() returns the same message.
 * The calls make the plan's device current while they run and restore the
 * caller's current device before returning.
 * ---------------------------------------------------------------------- */
typedef struct libm_hip_request {
  int fn;           /* libm_hip_fn */
  int variant;      /* libm_hip_variant */
  int dtype;        /* libm_hip_dtype */
  int reserved;
  const void* a;    /* first operand (C argument order) */
  const void* b;    /* second operand, NULL for unary functions */
  void* out;
  size_t n;
} libm_hip_request;
typedef struct libm_hip_batch_plan libm_hip_batch_plan;

libm_hip_status libm_hip_batch_plan_create(libm_hip_batch_plan** plan, int max_requests,
                                           int device);
libm_hip_status libm_hip_batch_plan_set_graph(libm_hip_batch_plan* plan, int use_graph);
libm_hip_status libm_hip_batch_run(libm_hip_batch_plan* plan, const libm_hip_request* requests,
                                   int k, void* stream);
void libm_hip_batch_plan_destroy(libm_hip_batch_plan* plan);
const char* libm_hip_batch_last_error(void);

/* ------------------------------------------------------------------------
 * The batched evaluation without any allocation, for callers that cannot
 * allocate device memory (code being captured into a hip graph, tight
 * serving loops, harnesses that forbid hipMalloc): the results of
 * libm_hip_batch_run (same kernels, same tile order) with no plan.  The
 * request table (at most 256 requests), its header and the tile counter
 * live in a fixed 12.5 KiB device array of the library, one per GPU, held
 * until the process ends; the table reaches it through a small staging
 * kernel that takes the requests as kernel arguments (no host-to-device
 * copy), and that kernel also clears the counter.  The call makes no
 * hipMalloc, hipFree or other allocating call.
 * Every call on one GPU uses that GPU's one array: calls that overlap on a
 * GPU (from several threads or on unordered streams) race and must be
 * ordered by the caller.  Arguments as libm_hip_batch_run, on the current
 * device's `stream`; LIBM_HIP_ERR_INVALID for k > 256 (message on
 * libm_hip_last_error), LIBM_HIP_ERR_UNSUPPORTED / LIBM_HIP_ERR_INVALID for
 * a bad request, LIBM_HIP_ERR_HIP for a launch failure.  Returns without
 * waiting for the kernels.
 * ---------------------------------------------------------------------- */
libm_hip_status libm_hip_batch_run_noalloc(const libm_hip_request* requests, int k,
                                           void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LIBM_HIP_H */
