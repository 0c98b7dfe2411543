// Element storage types and operation tags shared by the elementwise kernels
// (kernels.hip) and the batched persistent kernel (batch.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eval_f64.h"
#include "eval_f32.h"
#include "eval_half.h"
#include "eval_grad.h"
#pragma STDC FP_CONTRACT OFF

namespace lmh_ops {

// ---------------------------------------------------------------------------
// storage <-> compute conversions
// ---------------------------------------------------------------------------
struct IoF64 {
  typedef double S;
  typedef double C;
  static __device__ __forceinline__ C in(S v) { return v; }
  static __device__ __forceinline__ S out(C v) { return v; }
};
struct IoF32 {
  typedef float S;
  typedef float C;
  static __device__ __forceinline__ C in(S v) { return v; }
  static __device__ __forceinline__ S out(C v) { return v; }
};
// binary32 storage evaluated in binary64, rounded once
struct IoF32ViaF64 {
  typedef float S;
  typedef double C;
  static __device__ __forceinline__ C in(S v) { return (double)v; }
  static __device__ __forceinline__ S out(C v) { return (float)v; }
};
// bfloat16 bit patterns: widening is a shift; narrowing rounds to nearest
// even (NaN stays a quiet NaN)
struct IoBF16 {
  typedef uint16_t S;
  typedef float C;
  static __device__ __forceinline__ C in(S v) { return lmh::as_f32((int32_t)((uint32_t)v << 16)); }
  static __device__ __forceinline__ S out(C v) {
    uint32_t u = (uint32_t)lmh::as_i32(v);
    uint32_t r = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
    return (uint16_t)(lmh::isnan_(v) ? ((u >> 16) | 0x40u) : r);
  }
};
// IEEE binary16 bit patterns: hardware conversions (exact widening, RNE
// narrowing with overflow to inf and gradual underflow)
struct IoF16 {
  typedef uint16_t S;
  typedef float C;
  static __device__ __forceinline__ C in(S v) { return (float)__builtin_bit_cast(_Float16, v); }
  static __device__ __forceinline__ S out(C v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
};

// ---------------------------------------------------------------------------
// operation tags: one per evaluator, overloaded on the compute type
// ---------------------------------------------------------------------------
#define LMH_OP1(NAME, F64FN, F32FN)                                              \
  struct NAME {                                                                \
    static constexpr bool kSplit = false;                                      \
    static __device__ __forceinline__ double f(double x) { return lmh::F64FN(x); } \
    static __device__ __forceinline__ float f(float x) { return lmh::F32FN(x); }   \
  };
// tags of evaluators with a rare accurate path (results in the subnormal
// range): main(x, rare) is the common path and flags the lanes that need
// rare(x); f(x) does both.  The elementwise kernels evaluate main for a whole
// pack and then rare once for the flagged elements.
#define LMH_OP1R(NAME, F64FN, F32FN)                                                         \
  struct NAME {                                                                            \
    static constexpr bool kSplit = false;                                                  \
    static constexpr bool kRare = true;                                                    \
    static __device__ __forceinline__ double f(double x) { return lmh::F64FN(x); }         \
    static __device__ __forceinline__ float f(float x) { return lmh::F32FN(x); }           \
    static __device__ __forceinline__ double main(double x, bool& r) { return lmh::F64FN##_main(x, r); } \
    static __device__ __forceinline__ float main(float x, bool& r) { return lmh::F32FN##_main(x, r); }   \
    static __device__ __forceinline__ double rare(double x) { return lmh::F64FN##_rare(x); }  \
    static __device__ __forceinline__ float rare(float x) { return lmh::F32FN##_rare(x); }    \
  };
#define LMH_OP2R(NAME, F64FN, F32FN)                                                         \
  struct NAME {                                                                            \
    static constexpr bool kRare = true;                                                    \
    static __device__ __forceinline__ double f(double a, double b) { return lmh::F64FN(a, b); } \
    static __device__ __forceinline__ float f(float a, float b) { return lmh::F32FN(a, b); }    \
    static __device__ __forceinline__ double main(double a, double b, bool& r) {           \
      return lmh::F64FN##_main(a, b, r);                                                   \
    }                                                                                      \
    static __device__ __forceinline__ float main(float a, float b, bool& r) {              \
      return lmh::F32FN##_main(a, b, r);                                                   \
    }                                                                                      \
    static __device__ __forceinline__ double rare(double a, double b) { return lmh::F64FN##_rare(a, b); } \
    static __device__ __forceinline__ float rare(float a, float b) { return lmh::F32FN##_rare(a, b); }    \
  };
#define LMH_OP2(NAME, F64FN, F32FN)                                                        \
  struct NAME {                                                                          \
    static __device__ __forceinline__ double f(double a, double b) { return lmh::F64FN(a, b); } \
    static __device__ __forceinline__ float f(float a, float b) { return lmh::F32FN(a, b); }    \
  };

// Trigonometric tags also expose their reduction paths, so a kernel can
// gather the elements that need Payne-Hanek and run them densely:
// is_slow(x), fast(x) / slow(x) -> reduced state, finish(x, state) ->
// result.  Every route gives the bits of f(x).
#define LMH_TRIG_OP(NAME, F64FN, F32FN, RED64, RED32, ARG, FIN64, FIN32)                        \
  struct NAME {                                                                                 \
    static constexpr bool kSplit = true;                                                        \
    static __device__ __forceinline__ double f(double x) { return lmh::F64FN(x); }              \
    static __device__ __forceinline__ float f(float x) { return lmh::F32FN(x); }                \
    static __device__ __forceinline__ bool is_slow(double x) { return lmh::trig_slow(x); }      \
    static __device__ __forceinline__ bool is_slow(float x) { return lmh::trigf_slow(x); }      \
    static __device__ __forceinline__ lmh::Trig64 fast(double x) { return lmh::RED64##_fast(x ARG); } \
    static __device__ __forceinline__ lmh::Trig32 fast(float x) { return lmh::RED32##_fast(x ARG); }  \
    static __device__ __forceinline__ lmh::Trig64 slow(double x) { return lmh::RED64##_slow(x ARG); } \
    static __device__ __forceinline__ lmh::Trig32 slow(float x) { return lmh::RED32##_slow(x ARG); }  \
    static __device__ __forceinline__ double finish(double x, lmh::Trig64 s) { return lmh::FIN64(x, s); } \
    static __device__ __forceinline__ float finish(float x, lmh::Trig32 s) { return lmh::FIN32(x, s); }   \
  };
// sincos: fast(x) -> both reduction states, slow(x) -> the raw Payne-Hanek
// pair and quadrant, lift(x, raw) -> both states, finish_sin / finish_cos
#define LMH_SINCOS_OP(NAME, SFIN64, CFIN64, SFIN32, CFIN32)                                      \
  struct NAME {                                                                                 \
    static __device__ __forceinline__ bool is_slow(double x) { return lmh::trig_slow(x); }      \
    static __device__ __forceinline__ bool is_slow(float x) { return lmh::trigf_slow(x); }      \
    static __device__ __forceinline__ lmh::SinCos64 fast(double x) { return lmh::sincos2_fast(x); } \
    static __device__ __forceinline__ lmh::SinCos32 fast(float x) { return lmh::sincosf2_fast(x); } \
    static __device__ __forceinline__ lmh::Trig64 slow(double x) { return lmh::sincos_raw(x); }  \
    static __device__ __forceinline__ lmh::Trig32 slow(float x) { return lmh::sincosf_raw(x); }  \
    static __device__ __forceinline__ lmh::SinCos64 lift(double x, lmh::Trig64 r) {             \
      return lmh::sincos_lift(x, r);                                                            \
    }                                                                                           \
    static __device__ __forceinline__ lmh::SinCos32 lift(float x, lmh::Trig32 r) {              \
      return lmh::sincosf_lift(x, r);                                                           \
    }                                                                                           \
    static __device__ __forceinline__ double finish_sin(double x, lmh::SinCos64 s) {            \
      return lmh::SFIN64(x, s.s);                                                               \
    }                                                                                           \
    static __device__ __forceinline__ double finish_cos(double x, lmh::SinCos64 s) {            \
      return lmh::CFIN64(x, s.c);                                                               \
    }                                                                                           \
    static __device__ __forceinline__ float finish_sin(float x, lmh::SinCos32 s) {              \
      return lmh::SFIN32(x, s.s);                                                               \
    }                                                                                           \
    static __device__ __forceinline__ float finish_cos(float x, lmh::SinCos32 s) {              \
      return lmh::CFIN32(x, s.c);                                                               \
    }                                                                                           \
    /* one-call form (device API): both under the execution mask */                             \
    static __device__ __forceinline__ void f(double x, double& s, double& c) {                  \
      lmh::SinCos64 st = lmh::sincos2_reduce(x);                                                \
      s = lmh::SFIN64(x, st.s);                                                                 \
      c = lmh::CFIN64(x, st.c);                                                                 \
    }                                                                                           \
    static __device__ __forceinline__ void f(float x, float& s, float& c) {                     \
      lmh::SinCos32 st = lmh::sincosf2_reduce(x);                                               \
      s = lmh::SFIN32(x, st.s);                                                                 \
      c = lmh::CFIN32(x, st.c);                                                                 \
    }                                                                                           \
  };
LMH_SINCOS_OP(OpSinCosU10, sin_finish_u10, cos_finish_u10, sinf_finish_u10, cosf_finish_u10)
LMH_SINCOS_OP(OpSinCosU35, sin_finish_u35, cos_finish_u35, sinf_finish_u35, cosf_finish_u35)

#define LMH_NOARG
#define LMH_COMMA ,
LMH_TRIG_OP(OpSinU10, sin_u10, sinf_u10, sincos, sincosf, LMH_COMMA false, sin_finish_u10, sinf_finish_u10)
LMH_TRIG_OP(OpSinU35, sin_u35, sinf_u35, sincos, sincosf, LMH_COMMA false, sin_finish_u35, sinf_finish_u35)
LMH_TRIG_OP(OpCosU10, cos_u10, cosf_u10, sincos, sincosf, LMH_COMMA true, cos_finish_u10, cosf_finish_u10)
LMH_TRIG_OP(OpCosU35, cos_u35, cosf_u35, sincos, sincosf, LMH_COMMA true, cos_finish_u35, cosf_finish_u35)
LMH_TRIG_OP(OpTanU10, tan_u10, tanf_u10, tan, tanf, LMH_NOARG, tan_finish_u10, tanf_finish_u10)
LMH_TRIG_OP(OpTanU35, tan_u35, tanf_u35, tan, tanf, LMH_NOARG, tan_finish_u35, tanf_finish_u35)
LMH_OP1R(OpExpU10, exp_u10, expf_u10)
LMH_OP1R(OpExp2U10, exp2_u10, exp2f_u10)
LMH_OP1(OpLogU10, log_u10, logf_u10)
LMH_OP1(OpLogU35, log_u35, logf_u35)
LMH_OP1(OpLog2U10, log2_u10, log2f_u10)
LMH_OP1(OpSinhU10, sinh_u10, sinhf_u10)
LMH_OP1(OpCoshU10, cosh_u10, coshf_u10)
LMH_OP1(OpTanhU10, tanh_u10, tanhf_u10)
LMH_OP1(OpAsinU10, asin_u10, asinf_u10)
LMH_OP1(OpAsinU35, asin_u35, asinf_u35)
LMH_OP1(OpAcosU10, acos_u10, acosf_u10)
LMH_OP1(OpAcosU35, acos_u35, acosf_u35)
LMH_OP1(OpAtanU10, atan_u10, atanf_u10)
LMH_OP1(OpAtanU35, atan_u35, atanf_u35)
LMH_OP1(OpLog10U10, log10_u10, log10f_u10)
LMH_OP1(OpLog1pU10, log1p_u10, log1pf_u10)
LMH_OP1R(OpExp10U10, exp10_u10, exp10f_u10)
LMH_OP1(OpExpm1U10, expm1_u10, expm1f_u10)
LMH_OP1(OpCbrtU10, cbrt_u10, cbrtf_u10)
LMH_OP1(OpAsinhU10, asinh_u10, asinhf_u10)
LMH_OP1(OpAcoshU10, acosh_u10, acoshf_u10)
LMH_OP1(OpAtanhU10, atanh_u10, atanhf_u10)
LMH_OP1R(OpErfU10, erf_u10, erff_u10)
LMH_OP1R(OpErfcU10, erfc_u10, erfcf_u10)
LMH_OP1(OpLgammaU10, lgamma_u10, lgammaf_u10)
LMH_OP1R(OpTgammaU10, tgamma_u10, tgammaf_u10)
LMH_OP2R(OpHypotU10, hypot_u10, hypotf_u10)
LMH_OP1(OpSinhU35, sinh_u35, sinhf_u35)
LMH_OP1(OpCoshU35, cosh_u35, coshf_u35)
LMH_OP1(OpTanhU35, tanh_u35, tanhf_u35)
LMH_OP2R(OpAtan2U35, atan2_u35, atan2f_u35)
LMH_OP2R(OpPowU10, pow_u10, powf_u10)
LMH_OP2R(OpPowU35, pow_u35, powf_u35)
LMH_OP2(OpAtan2U10, atan2_u10, atan2f_u10)
LMH_OP2(OpFmod, fmod_f64, fmodf_f32)
LMH_OP2(OpRemainder, remainder_f64, remainderf_f32)
LMH_OP2(OpFdim, fdim_f64, fdimf_f32)
LMH_OP2(OpFmax, fmax_f64, fmaxf_f32)
LMH_OP2(OpFmin, fmin_f64, fminf_f32)
LMH_OP1(OpSqrt, sqrt_f64, sqrtf_f32)
LMH_OP1(OpTrunc, trunc_f64, truncf_f32)
LMH_OP1(OpFloor, floor_f64, floorf_f32)
LMH_OP1(OpCeil, ceil_f64, ceilf_f32)
LMH_OP1(OpRound, round_f64, roundf_f32)
LMH_OP1(OpRint, rint_f64, rintf_f32)
LMH_OP1(OpFabs, fabs_f64, fabsf_f32)
LMH_OP1(OpLogb, logb_f64, logbf_f32)
LMH_OP2(OpCopysign, copysign_f64, copysignf_f32)
LMH_OP2(OpNextafter, nextafter_f64, nextafterf_f32)
// the integer-operand functions
struct OpIntFns {
  static __device__ __forceinline__ double ldexp(double x, int n) { return lmh::ldexp_f64(x, n); }
  static __device__ __forceinline__ float ldexp(float x, int n) { return lmh::ldexpf_f32(x, n); }
  static __device__ __forceinline__ int ilogb(double x) { return lmh::ilogb_f64(x); }
  static __device__ __forceinline__ int ilogb(float x) { return lmh::ilogbf_f32(x); }
  static __device__ __forceinline__ double frexp_mant(double x) { return lmh::frexp_mant_f64(x); }
  static __device__ __forceinline__ float frexp_mant(float x) { return lmh::frexp_mantf_f32(x); }
  static __device__ __forceinline__ int frexp_exp(double x) { return lmh::frexp_exp_f64(x); }
  static __device__ __forceinline__ int frexp_exp(float x) { return lmh::frexp_expf_f32(x); }
  static __device__ __forceinline__ double modf_frac(double x) { return lmh::modf_frac_f64(x); }
  static __device__ __forceinline__ float modf_frac(float x) { return lmh::modf_fracf_f32(x); }
  static __device__ __forceinline__ double modf_int(double x) { return lmh::modf_int_f64(x); }
  static __device__ __forceinline__ float modf_int(float x) { return lmh::modf_intf_f32(x); }
  static __device__ __forceinline__ double fma(double x, double y, double z) { return lmh::fma_f64(x, y, z); }
  static __device__ __forceinline__ float fma(float x, float y, float z) { return lmh::fmaf_f32(x, y, z); }
  static __device__ __forceinline__ long long lrint(double x) { return lmh::lrint_f64(x); }
  static __device__ __forceinline__ long long lrint(float x) { return lmh::lrintf_f32(x); }
  static __device__ __forceinline__ long long lround(double x) { return lmh::lround_f64(x); }
  static __device__ __forceinline__ long long lround(float x) { return lmh::lroundf_f32(x); }
  static __device__ __forceinline__ double remquo_rem(double x, double y) { return lmh::remainder_f64(x, y); }
  static __device__ __forceinline__ float remquo_rem(float x, float y) { return lmh::remainderf_f32(x, y); }
  static __device__ __forceinline__ int remquo_quo(double x, double y) { return lmh::remquo_quo_f64(x, y); }
  static __device__ __forceinline__ int remquo_quo(float x, float y) { return lmh::remquo_quof_f32(x, y); }
};

// backward tags: (x, g) -> g f'(x); (a, b, g) -> two partials
#define LMH_OPB(NAME, FN)                                                                   \
  struct NAME {                                                                           \
    static __device__ __forceinline__ double f(double x, double g) { return lmh::FN(x, g); } \
    static __device__ __forceinline__ float f(float x, float g) { return lmh::FN(x, g); }    \
  };
LMH_OPB(OpSinBwd, sin_bwd)
LMH_OPB(OpCosBwd, cos_bwd)
LMH_OPB(OpTanBwd, tan_bwd)
LMH_OPB(OpExpBwd, exp_bwd)
LMH_OPB(OpLogBwd, log_bwd)
LMH_OPB(OpTanhBwd, tanh_bwd)
struct OpPowBwd {
  template <class T>
  static __device__ __forceinline__ void f(T x, T y, T g, T& gx, T& gy) { lmh::pow_bwd(x, y, g, gx, gy); }
};
struct OpAtan2Bwd {
  template <class T>
  static __device__ __forceinline__ void f(T y, T x, T g, T& gy, T& gx) { lmh::atan2_bwd(y, x, g, gy, gx); }
};


// 16 bytes of one operand for one lane; moved as a 128-bit vector so that the
// store can carry the non-temporal hint (the elements are touched once)
template <class S, int EPT>
struct alignas(16) Pack {
  S v[EPT];
};
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class P>
__device__ __forceinline__ void store_nt(const P& v, void* dst) {
  static_assert(sizeof(P) == 16, "one 128-bit store per lane");
  __builtin_nontemporal_store(__builtin_bit_cast(u32x4, v), reinterpret_cast<u32x4*>(dst));
}

// elements per lane and pack: 16 bytes of storage per lane and operand
template <class S>
constexpr int ept_for() { return 16 / (int)sizeof(S); }

// Evaluators of the narrow formats (eval_half.h): binary32 only
#define LMH_OPN(NAME, FN)                                                            \
  struct NAME {                                                                    \
    static constexpr bool kSplit = false;                                          \
    static __device__ __forceinline__ float f(float x) { return lmh::FN(x); }      \
  };
LMH_OPN(OpNExp, nexp)
LMH_OPN(OpNExp2, nexp2)
LMH_OPN(OpNLog, nlog)
LMH_OPN(OpNLog2, nlog2)
LMH_OPN(OpNSinh, nsinh)
LMH_OPN(OpNCosh, ncosh)
LMH_OPN(OpNTanh, ntanh)
LMH_OPN(OpHSin, hsin)
LMH_OPN(OpHCos, hcos)
LMH_OPN(OpHTan, htan)
LMH_OPN(OpNAtan, natan)
LMH_OPN(OpNAsin, nasin)
LMH_OPN(OpNAcos, nacos)
#undef LMH_OPN
struct OpNPow {
  static __device__ __forceinline__ float f(float x, float y) { return lmh::npow(x, y); }
};
struct OpNAtan2 {
  static __device__ __forceinline__ float f(float y, float x) { return lmh::natan2(y, x); }
};
// bf16 trig: each lane takes the reduction its argument needs; the integer
// Payne-Hanek reduction is short enough that the plain kernel runs it
// without gathering those lanes
#define LMH_NTRIG_OP(NAME, FIN)                                                                  \
  struct NAME {                                                                                \
    static constexpr bool kSplit = false;                                                      \
    static __device__ __forceinline__ float f(float x) { return lmh::FIN(x, lmh::nbtrig_reduce(x)); } \
  };
LMH_NTRIG_OP(OpNSin, nsin_fin)
LMH_NTRIG_OP(OpNCos, ncos_fin)
LMH_NTRIG_OP(OpNTan, ntan_fin)
#undef LMH_NTRIG_OP
// sincos of the narrow formats in the split kernel's interface: the state of
// cos is sin's with the quadrant advanced by one inside ncos_fin, so the
// results are the bits of the sin and cos evaluators.  SLOW: whether the
// Payne-Hanek reduction is ever needed (bf16) or never (f16).
template <bool SLOW>
struct OpNSinCos {
  static __device__ __forceinline__ bool is_slow(float x) { return SLOW && lmh::nbtrig_slow(x); }
  static __device__ __forceinline__ lmh::SinCos32 fast(float x) {
    lmh::Trig32 s = lmh::hsincos_reduce(x);
    return lmh::SinCos32{s, s};
  }
  static __device__ __forceinline__ lmh::Trig32 slow(float x) { return lmh::nbtrig_big(x); }
  static __device__ __forceinline__ lmh::SinCos32 lift(float, lmh::Trig32 s) {
    return lmh::SinCos32{s, s};
  }
  static __device__ __forceinline__ float finish_sin(float x, lmh::SinCos32 s) {
    return lmh::nsin_fin(x, s.s);
  }
  static __device__ __forceinline__ float finish_cos(float x, lmh::SinCos32 s) {
    return lmh::ncos_fin(x, s.c);
  }
  static __device__ __forceinline__ void f(float x, float& s, float& c) {
    lmh::Trig32 st = SLOW ? lmh::nbtrig_reduce(x) : lmh::hsincos_reduce(x);
    s = lmh::nsin_fin(x, st);
    c = lmh::ncos_fin(x, st);
  }
};

// The evaluator an (element type, function) pair runs.  f32_via_f64 goes
// through binary64, bf16 and f16 through binary32: the wider type carries at
// least 13 more bits (bf16: 16, f16: 13, binary32 from binary64: 29), so its
// 3.5-ULP evaluator, rounded once, is within 0.5 + 3.5 * 2^-13 ULP of the
// exact result in the narrow format, inside the 1.0-ULP bound; it is used
// wherever it exists.  Where a narrow-format evaluator exists (eval_half.h),
// bf16 and f16 run that instead.  Every path (entry points, dispatcher,
// batched kernel, device API) maps through this, so they agree bit for bit.
template <class Io, class Op>
struct EvalOp {
  typedef Op type;
};
#define LMH_EVAL_AS(IO, OP, AS)                       \
  template <>                                         \
  struct EvalOp<IO, OP> {                             \
    typedef AS type;                                  \
  };
#define LMH_WIDE_AND_HALF(OP10, OP35, OPN)            \
  LMH_EVAL_AS(IoBF16, OP10, OPN)                      \
  LMH_EVAL_AS(IoF16, OP10, OPN)                       \
  LMH_EVAL_AS(IoF32ViaF64, OP10, OP35)
#define LMH_HALF_ONLY(OP10, OPN)                      \
  LMH_EVAL_AS(IoBF16, OP10, OPN)                      \
  LMH_EVAL_AS(IoF16, OP10, OPN)
// trig: f16 in a plain kernel (no element needs Payne-Hanek), bf16 in the
// split kernel
#define LMH_TRIG_EVAL(OP10, OP35, OPB, OPH)           \
  LMH_EVAL_AS(IoBF16, OP10, OPB)                      \
  LMH_EVAL_AS(IoF16, OP10, OPH)                       \
  LMH_EVAL_AS(IoF32ViaF64, OP10, OP35)
LMH_TRIG_EVAL(OpSinU10, OpSinU35, OpNSin, OpHSin)
LMH_TRIG_EVAL(OpCosU10, OpCosU35, OpNCos, OpHCos)
LMH_TRIG_EVAL(OpTanU10, OpTanU35, OpNTan, OpHTan)
LMH_TRIG_EVAL(OpSinCosU10, OpSinCosU35, OpNSinCos<true>, OpNSinCos<false>)
LMH_WIDE_AND_HALF(OpLogU10, OpLogU35, OpNLog)
LMH_WIDE_AND_HALF(OpSinhU10, OpSinhU35, OpNSinh)
LMH_WIDE_AND_HALF(OpCoshU10, OpCoshU35, OpNCosh)
LMH_WIDE_AND_HALF(OpTanhU10, OpTanhU35, OpNTanh)
LMH_HALF_ONLY(OpExpU10, OpNExp)
LMH_HALF_ONLY(OpExp2U10, OpNExp2)
LMH_HALF_ONLY(OpLog2U10, OpNLog2)
LMH_HALF_ONLY(OpPowU10, OpNPow)
LMH_WIDE_AND_HALF(OpAsinU10, OpAsinU35, OpNAsin)
LMH_WIDE_AND_HALF(OpAcosU10, OpAcosU35, OpNAcos)
LMH_WIDE_AND_HALF(OpAtanU10, OpAtanU35, OpNAtan)
LMH_WIDE_AND_HALF(OpAtan2U10, OpAtan2U35, OpNAtan2)
#undef LMH_WIDE_AND_HALF
#undef LMH_HALF_ONLY
#undef LMH_TRIG_EVAL
#undef LMH_EVAL_AS

}  // namespace lmh_ops

#pragma STDC FP_CONTRACT DEFAULT
