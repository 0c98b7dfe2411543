// Scalar primitives of the gfx950 vector ALU used by every evaluator.
//
// Each maps to one CDNA instruction (or a short fixed sequence): v_fma_f64,
// v_rndne_f64 (round to nearest even), v_trunc_f64, v_ldexp_f64,
// v_frexp_mant_f64 / v_frexp_exp_i32_f64 (exact for subnormals too),
// v_rcp_f64, and the float counterparts.  The paper builds its functions from
// the same small set -- FMA, round-to-integer, mantissa/exponent extraction
// and conditional moves (Section 3.1, sub-features) -- so the evaluators stay
// branch-free except where a wave may skip a whole path no lane needs.
//
// Two builds share the evaluators.  The default one uses the hardware
// reciprocal, reciprocal square root and log2/exp2 estimates as the starting
// points of Newton steps.  With LMH_BITWISE_CONSISTENT defined, every
// primitive is an IEEE operation with one defined result (division and square
// root correctly rounded, a seed for x^(-1/3) from FMAs only), so the same
// evaluator source gives the same bits wherever it is compiled: on the GPU
// and, with LMH_HOST_SCALAR also defined, as a plain C++ build for the host
// (the paper's bit-consistent functions, Section 3.3).
#pragma once
#include <stdint.h>

// The evaluators depend on exactly where products are rounded: every fused
// multiply-add is written out, and no other product may be contracted
// (honoured under the default -ffp-contract; an explicit
// -ffp-contract=fast overrides it and changes results).
#pragma STDC FP_CONTRACT OFF

#ifdef LMH_HOST_SCALAR
#include "prims_host.h"
#else

#define LMH_INLINE __device__ __forceinline__

namespace lmh {

LMH_INLINE double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
LMH_INLINE float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
LMH_INLINE double rint_(double x) { return __builtin_rint(x); }
LMH_INLINE float rint_(float x) { return __builtin_rintf(x); }
LMH_INLINE double trunc_(double x) { return __builtin_trunc(x); }
LMH_INLINE float trunc_(float x) { return __builtin_truncf(x); }
LMH_INLINE double fabs_(double x) { return __builtin_fabs(x); }
LMH_INLINE float fabs_(float x) { return __builtin_fabsf(x); }
LMH_INLINE double copysign_(double a, double b) { return __builtin_copysign(a, b); }
LMH_INLINE float copysign_(float a, float b) { return __builtin_copysignf(a, b); }
LMH_INLINE double ldexp_(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }
LMH_INLINE float ldexp_(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }
// mantissa in [0.5, 1) with the sign of x, exponent such that x = m * 2^e;
// for +-0, inf and NaN the mantissa is x itself and the exponent 0
LMH_INLINE double frexp_mant_(double x) { return __builtin_amdgcn_frexp_mant(x); }
LMH_INLINE float frexp_mant_(float x) { return __builtin_amdgcn_frexp_mantf(x); }
LMH_INLINE int frexp_exp_(double x) { return __builtin_amdgcn_frexp_exp(x); }
LMH_INLINE int frexp_exp_(float x) { return __builtin_amdgcn_frexp_expf(x); }
LMH_INLINE bool isnan_(double x) { return __builtin_isnan(x); }
LMH_INLINE bool isnan_(float x) { return __builtin_isnan(x); }
LMH_INLINE bool isinf_(double x) { return __builtin_isinf(x); }
LMH_INLINE bool isinf_(float x) { return __builtin_isinf(x); }
LMH_INLINE bool isfinite_(double x) { return __builtin_isfinite(x); }
LMH_INLINE bool isfinite_(float x) { return __builtin_isfinite(x); }

LMH_INLINE int64_t as_i64(double x) { return __builtin_bit_cast(int64_t, x); }
LMH_INLINE double as_f64(int64_t x) { return __builtin_bit_cast(double, x); }
LMH_INLINE int32_t as_i32(float x) { return __builtin_bit_cast(int32_t, x); }
LMH_INLINE float as_f32(int32_t x) { return __builtin_bit_cast(float, x); }

// the transcendental unit in binary32: v_exp_f32 (2^x), v_log_f32 (log2 x)
// and v_rcp_f32 (1/x), each within about one binary32 ulp.  Only the
// narrow-format evaluators use them as results (their error is far below a
// bf16 or f16 ulp, and every bf16 and f16 input is tested).  GPU build only:
// the host build of the evaluators never includes those evaluators.
LMH_INLINE float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }
LMH_INLINE float log2_hw(float x) { return __builtin_amdgcn_logf(x); }
LMH_INLINE float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }

// true if the predicate holds on any active lane of the wavefront (used only
// to end a loop once every lane is done; the loop body stays exec-masked)
LMH_INLINE bool any_lane(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

}  // namespace lmh
#endif  // LMH_HOST_SCALAR

namespace lmh {

// any_lane for a path that only rare arguments take (results in the
// subnormal range): the instruction counts of the common path
// (gen/count_ops.py, built with LMH_COUNT_COMMON_PATH) leave such paths out,
// since almost no wave runs them
#ifdef LMH_COUNT_COMMON_PATH
LMH_INLINE bool rare_lane(bool) { return false; }
#else
LMH_INLINE bool rare_lane(bool p) { return any_lane(p); }
#endif

// the neighbour of a positive finite x towards zero (x > 0, not subnormal 0)
LMH_INLINE double pred_(double x) { return as_f64(as_i64(x) - 1); }
LMH_INLINE float pred_(float x) { return as_f32(as_i32(x) - 1); }

#ifdef LMH_BITWISE_CONSISTENT
// 1/x and 1/sqrt(x) as correctly rounded IEEE operations (the callers' Newton
// steps then leave them unchanged or move them by the same defined amount)
LMH_INLINE double rcp_(double x) { return 1.0 / x; }
LMH_INLINE float rcp_(float x) { return 1.0f / x; }
LMH_INLINE double rsq_(double x) { return 1.0 / __builtin_sqrt(x); }
LMH_INLINE float rsq_(float x) { return 1.0f / __builtin_sqrtf(x); }
// a^(-1/3) for a in [0.5, 4) to about 2^-43: a = m 2^i with m in [0.5, 1)
// and i in {0, 1, 2}; (1.49978 - 0.513 m) is within 1.33 % of m^(-1/3),
// times 2^(-i/3), then three Newton steps z += z (1 - a z^3)/3 (each squares
// the relative error and doubles it)
LMH_INLINE double rcbrt_seed(double a) {
  double m = frexp_mant_(a);
  int i = frexp_exp_(a);
  double k = i == 0 ? 1.0 : (i == 1 ? 0x1.965fea53d6e3dp-1 : 0x1.428a2f98d728bp-1);
  double z = fma_(m, -0.513, 1.499777789099392) * k;
  for (int it = 0; it < 3; ++it) z = fma_(z * (1.0 / 3.0), fma_(-a, z * z * z, 1.0), z);
  return z;
}
// binary32: the same seed and two Newton steps (about 2^-21)
LMH_INLINE float rcbrt_seed(float a) {
  float m = frexp_mant_(a);
  int i = frexp_exp_(a);
  float k = i == 0 ? 1.0f : (i == 1 ? 0x1.965feap-1f : 0x1.428a30p-1f);
  float z = fma_(m, -0.513f, 1.4997778f) * k;
  for (int it = 0; it < 2; ++it) z = fma_(z * (1.0f / 3.0f), fma_(-a, z * z * z, 1.0f), z);
  return z;
}
#else
// hardware reciprocal estimate (refined by the callers with Newton steps)
LMH_INLINE double rcp_(double x) { return __builtin_amdgcn_rcp(x); }
LMH_INLINE float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
// hardware reciprocal square root estimate (refined by Newton steps)
LMH_INLINE double rsq_(double x) { return __builtin_amdgcn_rsq(x); }
LMH_INLINE float rsq_(float x) { return __builtin_amdgcn_rsqf(x); }
// a^(-1/3) for a in [0.5, 4) from the hardware base-2 logarithm and
// exponential estimates (v_log_f32, v_exp_f32; about 22 correct bits), the
// starting point of the callers' Newton steps
LMH_INLINE float rcbrt_seed(float a) {
  return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(a) * (-1.0f / 3.0f));
}
LMH_INLINE double rcbrt_seed(double a) { return (double)rcbrt_seed((float)a); }
#endif

}  // namespace lmh

#pragma STDC FP_CONTRACT DEFAULT
