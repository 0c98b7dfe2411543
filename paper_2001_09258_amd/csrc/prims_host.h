// The primitives of prims.h for a host (CPU) build of the evaluators, used
// only by the bit-consistent host library.  Each is the IEEE operation with
// the same defined result as its GPU counterpart: fused multiply-add, round
// to nearest even integer, exact scaling and mantissa/exponent extraction
// (with the GPU's conventions for zero, infinity and NaN).
#pragma once
#ifndef LMH_BITWISE_CONSISTENT
#error "the host build of the evaluators exists only in the bitwise-consistent form"
#endif
#include <cmath>
#include <cstdint>
#include <cstring>

#define LMH_INLINE static inline
#define __device__

namespace lmh {

LMH_INLINE double fma_(double a, double b, double c) { return std::fma(a, b, c); }
LMH_INLINE float fma_(float a, float b, float c) { return std::fmaf(a, b, c); }
// nearbyint rounds in the current mode, which the library requires to be
// round-to-nearest-even
LMH_INLINE double rint_(double x) { return std::nearbyint(x); }
LMH_INLINE float rint_(float x) { return std::nearbyintf(x); }
LMH_INLINE double trunc_(double x) { return std::trunc(x); }
LMH_INLINE float trunc_(float x) { return std::truncf(x); }
LMH_INLINE double fabs_(double x) { return std::fabs(x); }
LMH_INLINE float fabs_(float x) { return std::fabs(x); }
LMH_INLINE double copysign_(double a, double b) { return std::copysign(a, b); }
LMH_INLINE float copysign_(float a, float b) { return std::copysign(a, b); }
LMH_INLINE double ldexp_(double x, int e) { return std::ldexp(x, e); }
LMH_INLINE float ldexp_(float x, int e) { return std::ldexp(x, e); }
LMH_INLINE double frexp_mant_(double x) {
  if (!std::isfinite(x) || x == 0.0) return x;
  int e;
  return std::frexp(x, &e);
}
LMH_INLINE float frexp_mant_(float x) {
  if (!std::isfinite(x) || x == 0.0f) return x;
  int e;
  return std::frexp(x, &e);
}
LMH_INLINE int frexp_exp_(double x) {
  int e = 0;
  if (std::isfinite(x) && x != 0.0) std::frexp(x, &e);
  return e;
}
LMH_INLINE int frexp_exp_(float x) {
  int e = 0;
  if (std::isfinite(x) && x != 0.0f) std::frexp(x, &e);
  return e;
}
LMH_INLINE bool isnan_(double x) { return std::isnan(x); }
LMH_INLINE bool isnan_(float x) { return std::isnan(x); }
LMH_INLINE bool isinf_(double x) { return std::isinf(x); }
LMH_INLINE bool isinf_(float x) { return std::isinf(x); }
LMH_INLINE bool isfinite_(double x) { return std::isfinite(x); }
LMH_INLINE bool isfinite_(float x) { return std::isfinite(x); }

LMH_INLINE int64_t as_i64(double x) { int64_t r; std::memcpy(&r, &x, 8); return r; }
LMH_INLINE double as_f64(int64_t x) { double r; std::memcpy(&r, &x, 8); return r; }
LMH_INLINE int32_t as_i32(float x) { int32_t r; std::memcpy(&r, &x, 4); return r; }
LMH_INLINE float as_f32(int32_t x) { float r; std::memcpy(&r, &x, 4); return r; }

// one element at a time: a path is needed exactly when this element needs it
LMH_INLINE bool any_lane(bool p) { return p; }

}  // namespace lmh
