// The bit-consistent form of the elementwise functions on the GPU (the
// paper's bit-consistent functions, Section 3.3): the same evaluator source
// compiled with LMH_BITWISE_CONSISTENT, so that every primitive is an IEEE
// operation with a defined result (no hardware estimate), and every element
// takes its own path (no reduction depends on other lanes).  The results
// equal, bit for bit, those of the host build of the same source
// (host_scalar.cpp, libm_hip_host_eval).  One plain kernel per function: an
// element per lane, grid-stride.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>

#define LMH_BITWISE_CONSISTENT 1
// its own namespace, so its inline evaluators never meet the default
// build's ones of the same name in this library
#define lmh lmh_bc
#include "eval_f32.h"
#undef lmh
#include "abi_util.h"
#include "fn_table.h"
#include "../../include/libm_hip.h"

namespace lmh_bc_kernels {

constexpr int BLOCK = 256;

template <class T, class F>
__global__ __launch_bounds__(BLOCK) void k_bc_unary(const T* a, T* y, size_t n) {
  size_t stride = (size_t)gridDim.x * BLOCK;
  for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) y[i] = F::f(a[i]);
}

template <class T, class F>
__global__ __launch_bounds__(BLOCK) void k_bc_binary(const T* a, const T* b, T* y, size_t n) {
  size_t stride = (size_t)gridDim.x * BLOCK;
  for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride)
    y[i] = F::f(a[i], b[i]);
}

#define LMH_BC_TAG1(FN, V, F64, F32)                                                        \
  struct Bc_##FN##_##V {                                                                  \
    static __device__ __forceinline__ double f(double x) { return lmh_bc::F64(x); }       \
    static __device__ __forceinline__ float f(float x) { return lmh_bc::F32(x); }         \
  };
#define LMH_BC_TAG2(FN, V, F64, F32)                                                        \
  struct Bc_##FN##_##V {                                                                  \
    static __device__ __forceinline__ double f(double a, double b) { return lmh_bc::F64(a, b); } \
    static __device__ __forceinline__ float f(float a, float b) { return lmh_bc::F32(a, b); }    \
  };
LMH_CONSISTENT_UNARY(LMH_BC_TAG1)
LMH_CONSISTENT_BINARY(LMH_BC_TAG2)

inline unsigned grid_for(size_t n) {
  size_t b = (n + BLOCK - 1) / BLOCK;
  return (unsigned)(b < 65536 ? b : 65536);
}

inline libm_hip_status launched(const char* what) {
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) return LIBM_HIP_OK;
  char buf[200];
  snprintf(buf, sizeof(buf), "libm_hip_consistent_eval: %s launch failed: %s", what,
           hipGetErrorString(e));
  lmh_abi::set_error(buf);
  return LIBM_HIP_ERR_HIP;
}

template <class F>
libm_hip_status run1(libm_hip_dtype t, const void* a, void* y, size_t n, hipStream_t s) {
  unsigned g = grid_for(n);
  if (t == LIBM_HIP_F64)
    hipLaunchKernelGGL((k_bc_unary<double, F>), dim3(g), dim3(BLOCK), 0, s, (const double*)a,
                       (double*)y, n);
  else
    hipLaunchKernelGGL((k_bc_unary<float, F>), dim3(g), dim3(BLOCK), 0, s, (const float*)a,
                       (float*)y, n);
  return launched("unary");
}

template <class F>
libm_hip_status run2(libm_hip_dtype t, const void* a, const void* b, void* y, size_t n,
                     hipStream_t s) {
  unsigned g = grid_for(n);
  if (t == LIBM_HIP_F64)
    hipLaunchKernelGGL((k_bc_binary<double, F>), dim3(g), dim3(BLOCK), 0, s, (const double*)a,
                       (const double*)b, (double*)y, n);
  else
    hipLaunchKernelGGL((k_bc_binary<float, F>), dim3(g), dim3(BLOCK), 0, s, (const float*)a,
                       (const float*)b, (float*)y, n);
  return launched("binary");
}

}  // namespace lmh_bc_kernels

extern "C" libm_hip_status libm_hip_consistent_eval(libm_hip_fn fn, libm_hip_variant v,
                                                    libm_hip_dtype t, const void* a,
                                                    const void* b, void* out, size_t n,
                                                    void* stream) {
  using namespace lmh_bc_kernels;
  if (t != LIBM_HIP_F64 && t != LIBM_HIP_F32) {
    lmh_abi::set_error("libm_hip_consistent_eval: binary64 and binary32 only");
    return LIBM_HIP_ERR_UNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
#define LMH_BC_CASE1(FN, V, F64, F32)                                                        \
  if (fn == LIBM_HIP_##FN && v == LIBM_HIP_##V) {                                          \
    if (n == 0) return LIBM_HIP_OK;                                                        \
    if (!a || !out) {                                                                      \
      lmh_abi::set_error("libm_hip_consistent_eval: NULL pointer with n > 0");             \
      return LIBM_HIP_ERR_INVALID;                                                         \
    }                                                                                      \
    return run1<Bc_##FN##_##V>(t, a, out, n, s);                                           \
  }
#define LMH_BC_CASE2(FN, V, F64, F32)                                                        \
  if (fn == LIBM_HIP_##FN && v == LIBM_HIP_##V) {                                          \
    if (n == 0) return LIBM_HIP_OK;                                                        \
    if (!a || !b || !out) {                                                                \
      lmh_abi::set_error("libm_hip_consistent_eval: NULL pointer with n > 0");             \
      return LIBM_HIP_ERR_INVALID;                                                         \
    }                                                                                      \
    return run2<Bc_##FN##_##V>(t, a, b, out, n, s);                                        \
  }
  LMH_CONSISTENT_UNARY(LMH_BC_CASE1)
  LMH_CONSISTENT_BINARY(LMH_BC_CASE2)
  lmh_abi::set_error("libm_hip_consistent_eval: unsupported function/variant");
  return LIBM_HIP_ERR_UNSUPPORTED;
}
