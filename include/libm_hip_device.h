/* libm_hip_device.h -- the libm_hip evaluators as device functions.
 *
 * For HIP device code on gfx950 that wants to apply a math function inside
 * its own kernel (a fused epilogue such as GELU-tanh, softplus or rotary
 * embeddings) instead of launching the library's elementwise kernels.  The
 * functions are the ones every entry point of libm_hip.h runs, so a value
 * computed here is bit-identical to the entry point's result for the same
 * input.  The paper builds its library as vector functions that
 * vectorizing compilers call from user loops (Section 4, the vector
 * function ABI); on a GPU that role is played by inlinable device
 * functions.
 *
 * Usage: #include "libm_hip_device.h" in a .hip file and call, e.g.,
 *   double y = libm_hip_device::sin_u10(x);            // binary64, 1.0 ULP
 *   float  z = libm_hip_device::tanh_u10(v);           // binary32, 1.0 ULP
 *   float  w = libm_hip_device::exp_u10_via_f64(v);    // binary64 evaluation
 *   uint16_t h = libm_hip_device::log_u10_bf16(bits);  // bf16 bit patterns
 *
 * Compile with the default -ffp-contract (or =on / =off): the evaluator
 * headers switch contraction off for their own code and restore the
 * command-line mode at their end.  An explicit -ffp-contract=fast, or
 * -ffast-math, overrides that and voids the accuracy bounds.  Denormals must
 * not be flushed (the HIP default on gfx950).
 *
 * Every function is a pure function of its arguments: no memory, no state,
 * no errno or flags; special values follow C99 Annex F as the entry points
 * do.  Accuracy: *_u10 within 1.0 ULP, *_u35 within 3.5 ULP, fmod and
 * remainder exact; bf16/f16 forms evaluate in binary32 (with the evaluators
 * sized for those formats where they exist, else the 3.5-ULP binary32 one
 * where it exists) and _via_f64 forms in binary64 (with the 3.5-ULP
 * evaluator where one exists, which the extra bits of the wider type keep
 * within 0.5 + 3.5 * 2^-13 ULP of the narrow result), and round once; each
 * gives the bits of the corresponding entry point.
 * The *_bwd functions return the vector-Jacobian product g * f'(x) (two
 * partials for pow and atan2) as the backward entry points do.
 */
#ifndef LIBM_HIP_DEVICE_H
#define LIBM_HIP_DEVICE_H

#include <stdint.h>

#include "../paper_2001_09258_amd/csrc/ops.h"

namespace libm_hip_device {

#define LIBM_HIP_DEVICE_EVAL(IO, OP) lmh_ops::EvalOp<lmh_ops::IO, lmh_ops::OP>::type
#define LIBM_HIP_DEVICE_UNARY(NAME, OP)                                                   \
  __device__ __forceinline__ double NAME(double x) { return lmh_ops::OP::f(x); }            \
  __device__ __forceinline__ float NAME(float x) { return lmh_ops::OP::f(x); }              \
  __device__ __forceinline__ float NAME##_via_f64(float x) {                                \
    return lmh_ops::IoF32ViaF64::out(                                                       \
        LIBM_HIP_DEVICE_EVAL(IoF32ViaF64, OP)::f(lmh_ops::IoF32ViaF64::in(x)));              \
  }                                                                                       \
  __device__ __forceinline__ uint16_t NAME##_bf16(uint16_t x) {                             \
    return lmh_ops::IoBF16::out(LIBM_HIP_DEVICE_EVAL(IoBF16, OP)::f(lmh_ops::IoBF16::in(x))); \
  }                                                                                       \
  __device__ __forceinline__ uint16_t NAME##_f16(uint16_t x) {                              \
    return lmh_ops::IoF16::out(LIBM_HIP_DEVICE_EVAL(IoF16, OP)::f(lmh_ops::IoF16::in(x)));    \
  }

#define LIBM_HIP_DEVICE_UNARY_WIDE(NAME, OP)                                              \
  __device__ __forceinline__ double NAME(double x) { return lmh_ops::OP::f(x); }            \
  __device__ __forceinline__ float NAME(float x) { return lmh_ops::OP::f(x); }

#define LIBM_HIP_DEVICE_BINARY_WIDE(NAME, OP)                                             \
  __device__ __forceinline__ double NAME(double a, double b) { return lmh_ops::OP::f(a, b); } \
  __device__ __forceinline__ float NAME(float a, float b) { return lmh_ops::OP::f(a, b); }

#define LIBM_HIP_DEVICE_BINARY(NAME, OP)                                                  \
  __device__ __forceinline__ double NAME(double a, double b) { return lmh_ops::OP::f(a, b); } \
  __device__ __forceinline__ float NAME(float a, float b) { return lmh_ops::OP::f(a, b); }    \
  __device__ __forceinline__ float NAME##_via_f64(float a, float b) {                       \
    return lmh_ops::IoF32ViaF64::out(LIBM_HIP_DEVICE_EVAL(IoF32ViaF64, OP)::f(               \
        lmh_ops::IoF32ViaF64::in(a), lmh_ops::IoF32ViaF64::in(b)));                          \
  }                                                                                       \
  __device__ __forceinline__ uint16_t NAME##_bf16(uint16_t a, uint16_t b) {                 \
    return lmh_ops::IoBF16::out(                                                            \
        LIBM_HIP_DEVICE_EVAL(IoBF16, OP)::f(lmh_ops::IoBF16::in(a), lmh_ops::IoBF16::in(b))); \
  }                                                                                       \
  __device__ __forceinline__ uint16_t NAME##_f16(uint16_t a, uint16_t b) {                  \
    return lmh_ops::IoF16::out(                                                             \
        LIBM_HIP_DEVICE_EVAL(IoF16, OP)::f(lmh_ops::IoF16::in(a), lmh_ops::IoF16::in(b)));    \
  }

/* sin, cos, tan (Section 5, sin/cos and tan), exp, log (Section 5, exp and
   log), exp2, log2, sinh, cosh, tanh: 1.0-ULP forms */
LIBM_HIP_DEVICE_UNARY(sin_u10, OpSinU10)
LIBM_HIP_DEVICE_UNARY(cos_u10, OpCosU10)
LIBM_HIP_DEVICE_UNARY(tan_u10, OpTanU10)
LIBM_HIP_DEVICE_UNARY(exp_u10, OpExpU10)
LIBM_HIP_DEVICE_UNARY(exp2_u10, OpExp2U10)
LIBM_HIP_DEVICE_UNARY(log_u10, OpLogU10)
LIBM_HIP_DEVICE_UNARY(log2_u10, OpLog2U10)
LIBM_HIP_DEVICE_UNARY(sinh_u10, OpSinhU10)
LIBM_HIP_DEVICE_UNARY(cosh_u10, OpCoshU10)
LIBM_HIP_DEVICE_UNARY(tanh_u10, OpTanhU10)
/* asin, acos (Section 5, asin and acos), atan (Section 5, atan) */
LIBM_HIP_DEVICE_UNARY(asin_u10, OpAsinU10)
LIBM_HIP_DEVICE_UNARY(acos_u10, OpAcosU10)
LIBM_HIP_DEVICE_UNARY(atan_u10, OpAtanU10)
/* log10, log1p, exp10, expm1, cbrt, asinh, acosh, atanh, erf, erfc (C99
   functions of the paper's library) */
LIBM_HIP_DEVICE_UNARY(log10_u10, OpLog10U10)
LIBM_HIP_DEVICE_UNARY(log1p_u10, OpLog1pU10)
LIBM_HIP_DEVICE_UNARY(exp10_u10, OpExp10U10)
LIBM_HIP_DEVICE_UNARY(expm1_u10, OpExpm1U10)
LIBM_HIP_DEVICE_UNARY(cbrt_u10, OpCbrtU10)
LIBM_HIP_DEVICE_UNARY(asinh_u10, OpAsinhU10)
LIBM_HIP_DEVICE_UNARY(acosh_u10, OpAcoshU10)
LIBM_HIP_DEVICE_UNARY(atanh_u10, OpAtanhU10)
LIBM_HIP_DEVICE_UNARY(erf_u10, OpErfU10)
LIBM_HIP_DEVICE_UNARY(erfc_u10, OpErfcU10)
LIBM_HIP_DEVICE_UNARY(lgamma_u10, OpLgammaU10)
LIBM_HIP_DEVICE_UNARY(tgamma_u10, OpTgammaU10)
/* 3.5-ULP forms (binary64 and binary32) */
LIBM_HIP_DEVICE_UNARY_WIDE(sin_u35, OpSinU35)
LIBM_HIP_DEVICE_UNARY_WIDE(cos_u35, OpCosU35)
LIBM_HIP_DEVICE_UNARY_WIDE(tan_u35, OpTanU35)
LIBM_HIP_DEVICE_UNARY_WIDE(asin_u35, OpAsinU35)
LIBM_HIP_DEVICE_UNARY_WIDE(acos_u35, OpAcosU35)
LIBM_HIP_DEVICE_UNARY_WIDE(atan_u35, OpAtanU35)
LIBM_HIP_DEVICE_UNARY_WIDE(log_u35, OpLogU35)
LIBM_HIP_DEVICE_UNARY_WIDE(sinh_u35, OpSinhU35)
LIBM_HIP_DEVICE_UNARY_WIDE(cosh_u35, OpCoshU35)
LIBM_HIP_DEVICE_UNARY_WIDE(tanh_u35, OpTanhU35)
/* pow(x, y) (Section 5, pow) and atan2(y, x), C argument order */
LIBM_HIP_DEVICE_BINARY(pow_u10, OpPowU10)
LIBM_HIP_DEVICE_BINARY(atan2_u10, OpAtan2U10)
LIBM_HIP_DEVICE_BINARY(hypot_u10, OpHypotU10)
LIBM_HIP_DEVICE_BINARY_WIDE(atan2_u35, OpAtan2U35)
LIBM_HIP_DEVICE_BINARY_WIDE(pow_u35, OpPowU35)

/* sincos: *s = sin x, *c = cos x, bit-identical to sin_* and cos_* of the
   same variant and type */
__device__ __forceinline__ void sincos_u10(double x, double* s, double* c) {
  lmh_ops::OpSinCosU10::f(x, *s, *c);
}
__device__ __forceinline__ void sincos_u10(float x, float* s, float* c) {
  lmh_ops::OpSinCosU10::f(x, *s, *c);
}
__device__ __forceinline__ void sincos_u35(double x, double* s, double* c) {
  lmh_ops::OpSinCosU35::f(x, *s, *c);
}
__device__ __forceinline__ void sincos_u35(float x, float* s, float* c) {
  lmh_ops::OpSinCosU35::f(x, *s, *c);
}
__device__ __forceinline__ void sincos_u10_via_f64(float x, float* s, float* c) {
  double sd, cd;
  LIBM_HIP_DEVICE_EVAL(IoF32ViaF64, OpSinCosU10)::f(lmh_ops::IoF32ViaF64::in(x), sd, cd);
  *s = lmh_ops::IoF32ViaF64::out(sd);
  *c = lmh_ops::IoF32ViaF64::out(cd);
}
__device__ __forceinline__ void sincos_u10_bf16(uint16_t x, uint16_t* s, uint16_t* c) {
  float sf, cf;
  LIBM_HIP_DEVICE_EVAL(IoBF16, OpSinCosU10)::f(lmh_ops::IoBF16::in(x), sf, cf);
  *s = lmh_ops::IoBF16::out(sf);
  *c = lmh_ops::IoBF16::out(cf);
}
__device__ __forceinline__ void sincos_u10_f16(uint16_t x, uint16_t* s, uint16_t* c) {
  float sf, cf;
  LIBM_HIP_DEVICE_EVAL(IoF16, OpSinCosU10)::f(lmh_ops::IoF16::in(x), sf, cf);
  *s = lmh_ops::IoF16::out(sf);
  *c = lmh_ops::IoF16::out(cf);
}

/* fmod(x, y) and remainder(x, y), exact (Section 5, FP remainder, Algorithm 1) */
__device__ __forceinline__ double fmod(double x, double y) { return lmh_ops::OpFmod::f(x, y); }
__device__ __forceinline__ float fmod(float x, float y) { return lmh_ops::OpFmod::f(x, y); }
__device__ __forceinline__ double remainder(double x, double y) {
  return lmh_ops::OpRemainder::f(x, y);
}
__device__ __forceinline__ float remainder(float x, float y) {
  return lmh_ops::OpRemainder::f(x, y);
}
/* fdim, fmax, fmin (C99 F.9.9), exact; -0 ordered below +0 */
__device__ __forceinline__ double fdim(double x, double y) { return lmh_ops::OpFdim::f(x, y); }
__device__ __forceinline__ float fdim(float x, float y) { return lmh_ops::OpFdim::f(x, y); }
__device__ __forceinline__ double fmax(double x, double y) { return lmh_ops::OpFmax::f(x, y); }
__device__ __forceinline__ float fmax(float x, float y) { return lmh_ops::OpFmax::f(x, y); }
__device__ __forceinline__ double fmin(double x, double y) { return lmh_ops::OpFmin::f(x, y); }
__device__ __forceinline__ float fmin(float x, float y) { return lmh_ops::OpFmin::f(x, y); }
/* ldexp, ilogb, frexp (C99 7.12.6): as the entry points of libm_hip.h */
__device__ __forceinline__ double ldexp(double x, int n) { return lmh_ops::OpIntFns::ldexp(x, n); }
__device__ __forceinline__ float ldexp(float x, int n) { return lmh_ops::OpIntFns::ldexp(x, n); }
__device__ __forceinline__ int ilogb(double x) { return lmh_ops::OpIntFns::ilogb(x); }
__device__ __forceinline__ int ilogb(float x) { return lmh_ops::OpIntFns::ilogb(x); }
__device__ __forceinline__ double frexp(double x, int* e) {
  *e = lmh_ops::OpIntFns::frexp_exp(x);
  return lmh_ops::OpIntFns::frexp_mant(x);
}
__device__ __forceinline__ float frexp(float x, int* e) {
  *e = lmh_ops::OpIntFns::frexp_exp(x);
  return lmh_ops::OpIntFns::frexp_mant(x);
}
/* remquo, modf, fma, lrint, lround (C99): as the entry points of libm_hip.h */
__device__ __forceinline__ double remquo(double x, double y, int* q) {
  *q = lmh_ops::OpIntFns::remquo_quo(x, y);
  return lmh_ops::OpIntFns::remquo_rem(x, y);
}
__device__ __forceinline__ float remquo(float x, float y, int* q) {
  *q = lmh_ops::OpIntFns::remquo_quo(x, y);
  return lmh_ops::OpIntFns::remquo_rem(x, y);
}
__device__ __forceinline__ double modf(double x, double* ip) {
  *ip = lmh_ops::OpIntFns::modf_int(x);
  return lmh_ops::OpIntFns::modf_frac(x);
}
__device__ __forceinline__ float modf(float x, float* ip) {
  *ip = lmh_ops::OpIntFns::modf_int(x);
  return lmh_ops::OpIntFns::modf_frac(x);
}
__device__ __forceinline__ double fma(double x, double y, double z) { return lmh_ops::OpIntFns::fma(x, y, z); }
__device__ __forceinline__ float fma(float x, float y, float z) { return lmh_ops::OpIntFns::fma(x, y, z); }
__device__ __forceinline__ long long lrint(double x) { return lmh_ops::OpIntFns::lrint(x); }
__device__ __forceinline__ long long lrint(float x) { return lmh_ops::OpIntFns::lrint(x); }
__device__ __forceinline__ long long lround(double x) { return lmh_ops::OpIntFns::lround(x); }
__device__ __forceinline__ long long lround(float x) { return lmh_ops::OpIntFns::lround(x); }
/* the rest of the exact C99 set: sqrt (correctly rounded), trunc, floor, ceil,
   round, rint, fabs, logb, copysign, nextafter */
__device__ __forceinline__ double sqrt(double x) { return lmh_ops::OpSqrt::f(x); }
__device__ __forceinline__ float sqrt(float x) { return lmh_ops::OpSqrt::f(x); }
__device__ __forceinline__ double trunc(double x) { return lmh_ops::OpTrunc::f(x); }
__device__ __forceinline__ float trunc(float x) { return lmh_ops::OpTrunc::f(x); }
__device__ __forceinline__ double floor(double x) { return lmh_ops::OpFloor::f(x); }
__device__ __forceinline__ float floor(float x) { return lmh_ops::OpFloor::f(x); }
__device__ __forceinline__ double ceil(double x) { return lmh_ops::OpCeil::f(x); }
__device__ __forceinline__ float ceil(float x) { return lmh_ops::OpCeil::f(x); }
__device__ __forceinline__ double round(double x) { return lmh_ops::OpRound::f(x); }
__device__ __forceinline__ float round(float x) { return lmh_ops::OpRound::f(x); }
__device__ __forceinline__ double rint(double x) { return lmh_ops::OpRint::f(x); }
__device__ __forceinline__ float rint(float x) { return lmh_ops::OpRint::f(x); }
__device__ __forceinline__ double fabs(double x) { return lmh_ops::OpFabs::f(x); }
__device__ __forceinline__ float fabs(float x) { return lmh_ops::OpFabs::f(x); }
__device__ __forceinline__ double logb(double x) { return lmh_ops::OpLogb::f(x); }
__device__ __forceinline__ float logb(float x) { return lmh_ops::OpLogb::f(x); }
__device__ __forceinline__ double copysign(double x, double y) { return lmh_ops::OpCopysign::f(x, y); }
__device__ __forceinline__ float copysign(float x, float y) { return lmh_ops::OpCopysign::f(x, y); }
__device__ __forceinline__ double nextafter(double x, double y) { return lmh_ops::OpNextafter::f(x, y); }
__device__ __forceinline__ float nextafter(float x, float y) { return lmh_ops::OpNextafter::f(x, y); }

/* backward: g * f'(x) */
#define LIBM_HIP_DEVICE_BWD(NAME, FN)                                                     \
  __device__ __forceinline__ double NAME(double x, double g) { return lmh::FN(x, g); }      \
  __device__ __forceinline__ float NAME(float x, float g) { return lmh::FN(x, g); }
LIBM_HIP_DEVICE_BWD(sin_u10_bwd, sin_bwd)
LIBM_HIP_DEVICE_BWD(cos_u10_bwd, cos_bwd)
LIBM_HIP_DEVICE_BWD(tan_u10_bwd, tan_bwd)
LIBM_HIP_DEVICE_BWD(exp_u10_bwd, exp_bwd)
LIBM_HIP_DEVICE_BWD(log_u10_bwd, log_bwd)
LIBM_HIP_DEVICE_BWD(tanh_u10_bwd, tanh_bwd)
__device__ __forceinline__ void pow_u10_bwd(double x, double y, double g, double* gx, double* gy) {
  lmh::pow_bwd(x, y, g, *gx, *gy);
}
__device__ __forceinline__ void pow_u10_bwd(float x, float y, float g, float* gx, float* gy) {
  lmh::pow_bwd(x, y, g, *gx, *gy);
}
__device__ __forceinline__ void atan2_u10_bwd(double y, double x, double g, double* gy,
                                              double* gx) {
  lmh::atan2_bwd(y, x, g, *gy, *gx);
}
__device__ __forceinline__ void atan2_u10_bwd(float y, float x, float g, float* gy, float* gx) {
  lmh::atan2_bwd(y, x, g, *gy, *gx);
}

/* masked evaluation (a whole function computing only the elements an opmask
   selects, Section 3.1): lanes whose mask is false return their argument
   unchanged, and a wave whose lanes are all masked off skips the work */
template <class T, class F>
__device__ __forceinline__ T masked(bool active, T x, F f) {
  T r = x;
  if (active) r = f(x);
  return r;
}

#undef LIBM_HIP_DEVICE_UNARY
#undef LIBM_HIP_DEVICE_EVAL
#undef LIBM_HIP_DEVICE_UNARY_WIDE
#undef LIBM_HIP_DEVICE_BINARY
#undef LIBM_HIP_DEVICE_BINARY_WIDE
#undef LIBM_HIP_DEVICE_BWD

}  // namespace libm_hip_device

#endif /* LIBM_HIP_DEVICE_H */
