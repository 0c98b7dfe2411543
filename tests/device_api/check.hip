// Test helper (not part of the library): a kernel that evaluates through the
// device-callable API of include/libm_hip_device.h, built WITHOUT
// -ffp-contract=off so that the headers' own contraction control is what
// keeps the results identical to the library's entry points.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/libm_hip_device.h"

namespace {
namespace D = libm_hip_device;

template <class S, class F>
__global__ void k1(const S* a, S* y, size_t n, F f) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f(a[i]);
}
template <class S, class F>
__global__ void k2(const S* a, const S* b, S* y, size_t n, F f) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f(a[i], b[i]);
}
// masked: every other element keeps its input
template <class S, class F>
__global__ void km(const S* a, S* y, size_t n, F f) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = D::masked((i & 1) == 0, a[i], f);
}

template <class S, class F>
int launch1(const void* a, void* y, size_t n, void* s, F f) {
  unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL((k1<S, F>), dim3(g), dim3(256), 0, (hipStream_t)s, (const S*)a, (S*)y, n, f);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}
template <class S, class F>
int launch2(const void* a, const void* b, void* y, size_t n, void* s, F f) {
  unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL((k2<S, F>), dim3(g), dim3(256), 0, (hipStream_t)s, (const S*)a, (const S*)b,
                     (S*)y, n, f);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}
}  // namespace

// fn, variant, dtype use the codes of libm_hip.h's enums
#define U1(NAME)                                                                            \
  switch (dtype) {                                                                          \
    case 0: return launch1<double>(a, y, n, s, [] __device__(double x) { return D::NAME(x); }); \
    case 1: return launch1<float>(a, y, n, s, [] __device__(float x) { return D::NAME(x); });   \
    case 2: return launch1<uint16_t>(a, y, n, s, [] __device__(uint16_t x) { return D::NAME##_bf16(x); }); \
    case 3: return launch1<uint16_t>(a, y, n, s, [] __device__(uint16_t x) { return D::NAME##_f16(x); });  \
    case 4: return launch1<float>(a, y, n, s, [] __device__(float x) { return D::NAME##_via_f64(x); });    \
  }                                                                                         \
  return 2;
#define U1W(NAME)                                                                           \
  switch (dtype) {                                                                          \
    case 0: return launch1<double>(a, y, n, s, [] __device__(double x) { return D::NAME(x); }); \
    case 1: return launch1<float>(a, y, n, s, [] __device__(float x) { return D::NAME(x); });   \
  }                                                                                         \
  return 2;
#define B2(NAME)                                                                            \
  switch (dtype) {                                                                          \
    case 0: return launch2<double>(a, b, y, n, s, [] __device__(double u, double v) { return D::NAME(u, v); }); \
    case 1: return launch2<float>(a, b, y, n, s, [] __device__(float u, float v) { return D::NAME(u, v); });    \
    case 2: return launch2<uint16_t>(a, b, y, n, s, [] __device__(uint16_t u, uint16_t v) { return D::NAME##_bf16(u, v); }); \
    case 3: return launch2<uint16_t>(a, b, y, n, s, [] __device__(uint16_t u, uint16_t v) { return D::NAME##_f16(u, v); });  \
    case 4: return launch2<float>(a, b, y, n, s, [] __device__(float u, float v) { return D::NAME##_via_f64(u, v); });       \
  }                                                                                         \
  return 2;
#define U1W(NAME)                                                                           \
  switch (dtype) {                                                                          \
    case 0: return launch1<double>(a, y, n, s, [] __device__(double x) { return D::NAME(x); }); \
    case 1: return launch1<float>(a, y, n, s, [] __device__(float x) { return D::NAME(x); });   \
  }                                                                                         \
  return 2;
#define B2W(NAME)                                                                           \
  switch (dtype) {                                                                          \
    case 0: return launch2<double>(a, b, y, n, s, [] __device__(double u, double v) { return D::NAME(u, v); }); \
    case 1: return launch2<float>(a, b, y, n, s, [] __device__(float u, float v) { return D::NAME(u, v); });    \
  }                                                                                         \
  return 2;

extern "C" int device_api_eval(int fn, int variant, int dtype, const void* a, const void* b,
                               void* y, size_t n, void* s) {
  if (n == 0) return 0;
  if (variant == 1) {
    switch (fn) {
      case 0: U1W(sin_u35)
      case 1: U1W(cos_u35)
      case 2: U1W(tan_u35)
      case 14: U1W(asin_u35)
      case 15: U1W(acos_u35)
      case 16: U1W(atan_u35)
      case 5: U1W(log_u35)
      case 8: B2W(atan2_u35)
      case 7: B2W(pow_u35)
      case 9: U1W(sinh_u35)
      case 10: U1W(cosh_u35)
      case 11: U1W(tanh_u35)
    }
    return 2;
  }
  switch (fn) {
    case 0: U1(sin_u10)
    case 1: U1(cos_u10)
    case 2: U1(tan_u10)
    case 3: U1(exp_u10)
    case 4: U1(exp2_u10)
    case 5: U1(log_u10)
    case 6: U1(log2_u10)
    case 7: B2(pow_u10)
    case 8: B2(atan2_u10)
    case 9: U1(sinh_u10)
    case 10: U1(cosh_u10)
    case 11: U1(tanh_u10)
    case 12: B2W(fmod)
    case 13: B2W(remainder)
    case 14: U1(asin_u10)
    case 15: U1(acos_u10)
    case 16: U1(atan_u10)
    case 17: U1(log10_u10)
    case 18: U1(log1p_u10)
    case 19: U1(exp10_u10)
    case 20: U1(expm1_u10)
    case 21: U1(cbrt_u10)
    case 22: B2(hypot_u10)
    case 23: U1(asinh_u10)
    case 24: U1(acosh_u10)
    case 25: U1(atanh_u10)
    case 26: U1(erf_u10)
    case 27: U1(erfc_u10)
    case 41: U1(lgamma_u10)
    case 42: U1(tgamma_u10)
    case 28: B2W(fdim)
    case 29: B2W(fmax)
    case 30: B2W(fmin)
    case 31: U1W(sqrt)
    case 32: U1W(trunc)
    case 33: U1W(floor)
    case 34: U1W(ceil)
    case 35: U1W(round)
    case 36: U1W(rint)
    case 37: U1W(fabs)
    case 38: U1W(logb)
    case 39: B2W(copysign)
    case 40: B2W(nextafter)
  }
  return 2;
}

// sin u10 binary64 on the even elements only, the odd ones copied
extern "C" int device_api_masked_sin(const double* a, double* y, size_t n, void* s) {
  if (n == 0) return 0;
  unsigned g = (unsigned)((n + 255) / 256);
  auto f = [] __device__(double x) { return D::sin_u10(x); };
  hipLaunchKernelGGL((km<double, decltype(f)>), dim3(g), dim3(256), 0, (hipStream_t)s, a, y, n, f);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

// sincos through the device API: s and c outputs
template <class S, class F>
__global__ void ksc(const S* a, S* ys, S* yc, size_t n, F f) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f(a[i], &ys[i], &yc[i]);
}
template <class S, class F>
int launch_sc(const void* a, void* ys, void* yc, size_t n, void* s, F f) {
  unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL((ksc<S, F>), dim3(g), dim3(256), 0, (hipStream_t)s, (const S*)a, (S*)ys,
                     (S*)yc, n, f);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}

extern "C" int device_api_sincos(int variant, int dtype, const void* a, void* ys, void* yc,
                                 size_t n, void* s) {
  if (n == 0) return 0;
  if (variant == 1) {
    switch (dtype) {
      case 0: return launch_sc<double>(a, ys, yc, n, s, [] __device__(double x, double* p, double* q) { D::sincos_u35(x, p, q); });
      case 1: return launch_sc<float>(a, ys, yc, n, s, [] __device__(float x, float* p, float* q) { D::sincos_u35(x, p, q); });
    }
    return 2;
  }
  switch (dtype) {
    case 0: return launch_sc<double>(a, ys, yc, n, s, [] __device__(double x, double* p, double* q) { D::sincos_u10(x, p, q); });
    case 1: return launch_sc<float>(a, ys, yc, n, s, [] __device__(float x, float* p, float* q) { D::sincos_u10(x, p, q); });
    case 2: return launch_sc<uint16_t>(a, ys, yc, n, s, [] __device__(uint16_t x, uint16_t* p, uint16_t* q) { D::sincos_u10_bf16(x, p, q); });
    case 3: return launch_sc<uint16_t>(a, ys, yc, n, s, [] __device__(uint16_t x, uint16_t* p, uint16_t* q) { D::sincos_u10_f16(x, p, q); });
    case 4: return launch_sc<float>(a, ys, yc, n, s, [] __device__(float x, float* p, float* q) { D::sincos_u10_via_f64(x, p, q); });
  }
  return 2;
}
