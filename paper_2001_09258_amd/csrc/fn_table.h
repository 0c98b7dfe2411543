// Every (function, variant) of the bit-consistent builds with its binary64
// and binary32 evaluators: X(FN, VARIANT, binary64 evaluator, binary32
// evaluator), FN and VARIANT naming libm_hip_fn and libm_hip_variant values
// without their LIBM_HIP_ prefix.  The GPU build (consistent.hip) and the
// host build (host_scalar.cpp) expand the same lists.
#pragma once

#define LMH_CONSISTENT_UNARY(X)                                                       \
  X(SIN, U10, sin_u10, sinf_u10) X(SIN, U35, sin_u35, sinf_u35)                       \
  X(COS, U10, cos_u10, cosf_u10) X(COS, U35, cos_u35, cosf_u35)                       \
  X(TAN, U10, tan_u10, tanf_u10) X(TAN, U35, tan_u35, tanf_u35)                       \
  X(EXP, U10, exp_u10, expf_u10) X(EXP2, U10, exp2_u10, exp2f_u10)                    \
  X(LOG, U10, log_u10, logf_u10) X(LOG, U35, log_u35, logf_u35)                       \
  X(LOG2, U10, log2_u10, log2f_u10)                                                   \
  X(SINH, U10, sinh_u10, sinhf_u10) X(SINH, U35, sinh_u35, sinhf_u35)                 \
  X(COSH, U10, cosh_u10, coshf_u10) X(COSH, U35, cosh_u35, coshf_u35)                 \
  X(TANH, U10, tanh_u10, tanhf_u10) X(TANH, U35, tanh_u35, tanhf_u35)                 \
  X(ASIN, U10, asin_u10, asinf_u10) X(ASIN, U35, asin_u35, asinf_u35)                 \
  X(ACOS, U10, acos_u10, acosf_u10) X(ACOS, U35, acos_u35, acosf_u35)                 \
  X(ATAN, U10, atan_u10, atanf_u10) X(ATAN, U35, atan_u35, atanf_u35)                 \
  X(LOG10, U10, log10_u10, log10f_u10) X(LOG1P, U10, log1p_u10, log1pf_u10)           \
  X(EXP10, U10, exp10_u10, exp10f_u10) X(EXPM1, U10, expm1_u10, expm1f_u10)           \
  X(CBRT, U10, cbrt_u10, cbrtf_u10)                                                   \
  X(ASINH, U10, asinh_u10, asinhf_u10) X(ACOSH, U10, acosh_u10, acoshf_u10)           \
  X(ATANH, U10, atanh_u10, atanhf_u10)                                                \
  X(ERF, U10, erf_u10, erff_u10) X(ERFC, U10, erfc_u10, erfcf_u10)                   \
  X(LGAMMA, U10, lgamma_u10, lgammaf_u10) X(TGAMMA, U10, tgamma_u10, tgammaf_u10)    \
  X(SQRT, EXACT, sqrt_f64, sqrtf_f32) X(TRUNC, EXACT, trunc_f64, truncf_f32)         \
  X(FLOOR, EXACT, floor_f64, floorf_f32) X(CEIL, EXACT, ceil_f64, ceilf_f32)         \
  X(ROUND, EXACT, round_f64, roundf_f32) X(RINT, EXACT, rint_f64, rintf_f32)         \
  X(FABS, EXACT, fabs_f64, fabsf_f32) X(LOGB, EXACT, logb_f64, logbf_f32)

#define LMH_CONSISTENT_BINARY(X)                                                      \
  X(POW, U10, pow_u10, powf_u10) X(POW, U35, pow_u35, powf_u35)                       \
  X(ATAN2, U10, atan2_u10, atan2f_u10) X(ATAN2, U35, atan2_u35, atan2f_u35)           \
  X(HYPOT, U10, hypot_u10, hypotf_u10)                                                \
  X(FMOD, EXACT, fmod_f64, fmodf_f32) X(REMAINDER, EXACT, remainder_f64, remainderf_f32)     \
  X(FDIM, EXACT, fdim_f64, fdimf_f32) X(FMAX, EXACT, fmax_f64, fmaxf_f32)                     \
  X(FMIN, EXACT, fmin_f64, fminf_f32) X(COPYSIGN, EXACT, copysign_f64, copysignf_f32)         \
  X(NEXTAFTER, EXACT, nextafter_f64, nextafterf_f32)
