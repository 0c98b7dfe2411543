// The host (CPU) build of the evaluators in their bit-consistent form: the
// same evaluator source as the GPU library, compiled by a C++ compiler with
// LMH_HOST_SCALAR and LMH_BITWISE_CONSISTENT, one element at a time.  Its
// results equal, bit for bit, those of libm_hip_consistent_eval on the GPU
// (the paper's bit-consistent functions, Section 3.3).  This is a separate
// library for callers that need the host to reproduce GPU results; no GPU
// entry point ever calls it.
//
// Build with round-to-nearest-even in effect and without floating-point
// contraction or reassociation (-ffp-contract=off, no -ffast-math).
#define LMH_HOST_SCALAR 1
#define LMH_BITWISE_CONSISTENT 1
#include <stddef.h>

#include "eval_f32.h"
#include "fn_table.h"
#include "../../include/libm_hip_host.h"

namespace {

template <class T, class F>
void map1(const void* a, void* y, size_t n, F f) {
  const T* x = (const T*)a;
  T* r = (T*)y;
  for (size_t i = 0; i < n; ++i) r[i] = f(x[i]);
}

template <class T, class F>
void map2(const void* a, const void* b, void* y, size_t n, F f) {
  const T* x = (const T*)a;
  const T* z = (const T*)b;
  T* r = (T*)y;
  for (size_t i = 0; i < n; ++i) r[i] = f(x[i], z[i]);
}

}  // namespace

extern "C" libm_hip_status libm_hip_host_eval(libm_hip_fn fn, libm_hip_variant v,
                                              libm_hip_dtype t, const void* a, const void* b,
                                              void* out, size_t n) {
  if (t != LIBM_HIP_F64 && t != LIBM_HIP_F32) return LIBM_HIP_ERR_UNSUPPORTED;
#define LMH_HOST_CASE1(FN, V, F64, F32)                                                      \
  if (fn == LIBM_HIP_##FN && v == LIBM_HIP_##V) {                                          \
    if (n == 0) return LIBM_HIP_OK;                                                        \
    if (!a || !out) return LIBM_HIP_ERR_INVALID;                                           \
    if (t == LIBM_HIP_F64)                                                                 \
      map1<double>(a, out, n, [](double x) { return lmh::F64(x); });                       \
    else                                                                                   \
      map1<float>(a, out, n, [](float x) { return lmh::F32(x); });                         \
    return LIBM_HIP_OK;                                                                    \
  }
#define LMH_HOST_CASE2(FN, V, F64, F32)                                                      \
  if (fn == LIBM_HIP_##FN && v == LIBM_HIP_##V) {                                          \
    if (n == 0) return LIBM_HIP_OK;                                                        \
    if (!a || !b || !out) return LIBM_HIP_ERR_INVALID;                                     \
    if (t == LIBM_HIP_F64)                                                                 \
      map2<double>(a, b, out, n, [](double x, double y) { return lmh::F64(x, y); });       \
    else                                                                                   \
      map2<float>(a, b, out, n, [](float x, float y) { return lmh::F32(x, y); });          \
    return LIBM_HIP_OK;                                                                    \
  }
  LMH_CONSISTENT_UNARY(LMH_HOST_CASE1)
  LMH_CONSISTENT_BINARY(LMH_HOST_CASE2)
  return LIBM_HIP_ERR_UNSUPPORTED;
}

extern "C" libm_hip_status libm_hip_host_fmod_steps(libm_hip_dtype t, const void* x,
                                                    const void* y, void* out, int32_t* steps,
                                                    size_t n) {
  if (t != LIBM_HIP_F64 && t != LIBM_HIP_F32) return LIBM_HIP_ERR_UNSUPPORTED;
  if (n == 0) return LIBM_HIP_OK;
  if (!x || !y || !out || !steps) return LIBM_HIP_ERR_INVALID;
  for (size_t i = 0; i < n; ++i) {
    int s = 0;
    if (t == LIBM_HIP_F64) {
      double a = ((const double*)x)[i], b = ((const double*)y)[i];
      double na = lmh::fabs_(a), nb = lmh::fabs_(b);
      if (lmh::isfinite_(a) && lmh::isfinite_(nb) && nb != 0.0 && na >= nb)
        lmh::fmod_core_steps(na, nb, s);
      ((double*)out)[i] = lmh::fmod_f64(a, b);
    } else {
      float a = ((const float*)x)[i], b = ((const float*)y)[i];
      float na = lmh::fabs_(a), nb = lmh::fabs_(b);
      if (lmh::isfinite_(a) && lmh::isfinite_(nb) && nb != 0.0f && na >= nb)
        lmh::fmodf_core_steps(na, nb, s);
      ((float*)out)[i] = lmh::fmodf_f32(a, b);
    }
    steps[i] = s;
  }
  return LIBM_HIP_OK;
}
