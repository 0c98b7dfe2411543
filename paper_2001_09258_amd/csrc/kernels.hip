// Elementwise kernels and the C-ABI of libm_hip.
//
// One lane evaluates EPT consecutive elements; a 256-lane workgroup covers
// 256*EPT elements.  Arrays whose pointers are all 16-byte aligned move data
// with 128-bit global loads and non-temporal 128-bit stores (the elements are
// touched once); any other alignment, and the ragged tail, use scalar
// accesses.  The per-element work is one evaluator from eval_f64.h /
// eval_f32.h: the paper's vector-of-lanes execution becomes one element per
// GPU lane, and its conditional moves become exec-masked selects.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "ops.h"
#include "../../include/libm_hip.h"

namespace {
using namespace lmh_ops;

thread_local char g_last_error[256] = "";

void set_error(const char* msg) {
  strncpy(g_last_error, msg, sizeof(g_last_error) - 1);
  g_last_error[sizeof(g_last_error) - 1] = 0;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
constexpr int BLOCK = 256;

// 16 bytes of one operand for one lane; moved as a 128-bit vector so that the
// store can carry the non-temporal hint
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

template <class Io, class Op, int EPT, bool VEC>
__global__ __launch_bounds__(BLOCK) void k_unary(const typename Io::S* __restrict__ x,
                                                 typename Io::S* __restrict__ y, size_t n) {
  typedef typename Io::S S;
  size_t base = ((size_t)blockIdx.x * BLOCK + threadIdx.x) * EPT;
  if (base >= n) return;
  if (VEC && base + EPT <= n) {
    Pack<S, EPT> in = *reinterpret_cast<const Pack<S, EPT>*>(x + base);
    Pack<S, EPT> out;
#pragma unroll
    for (int i = 0; i < EPT; ++i) out.v[i] = Io::out(Op::f(Io::in(in.v[i])));
    store_nt(out, y + base);
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      if (base + i < n) y[base + i] = Io::out(Op::f(Io::in(x[base + i])));
    }
  }
}

template <class Io, class Op, int EPT, bool VEC>
__global__ __launch_bounds__(BLOCK) void k_binary(const typename Io::S* __restrict__ a,
                                                  const typename Io::S* __restrict__ b,
                                                  typename Io::S* __restrict__ y, size_t n) {
  typedef typename Io::S S;
  size_t base = ((size_t)blockIdx.x * BLOCK + threadIdx.x) * EPT;
  if (base >= n) return;
  if (VEC && base + EPT <= n) {
    Pack<S, EPT> ia = *reinterpret_cast<const Pack<S, EPT>*>(a + base);
    Pack<S, EPT> ib = *reinterpret_cast<const Pack<S, EPT>*>(b + base);
    Pack<S, EPT> out;
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      out.v[i] = Io::out(Op::f(Io::in(ia.v[i]), Io::in(ib.v[i])));
    store_nt(out, y + base);
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      if (base + i < n) y[base + i] = Io::out(Op::f(Io::in(a[base + i]), Io::in(b[base + i])));
    }
  }
}

// three inputs, two outputs (backward of the binary functions)
template <class Io, class Op, int EPT, bool VEC>
__global__ __launch_bounds__(BLOCK) void k_ternary2(const typename Io::S* __restrict__ a,
                                                    const typename Io::S* __restrict__ b,
                                                    const typename Io::S* __restrict__ c,
                                                    typename Io::S* __restrict__ y0,
                                                    typename Io::S* __restrict__ y1, size_t n) {
  typedef typename Io::S S;
  typedef typename Io::C C;
  size_t base = ((size_t)blockIdx.x * BLOCK + threadIdx.x) * EPT;
  if (base >= n) return;
  if (VEC && base + EPT <= n) {
    Pack<S, EPT> ia = *reinterpret_cast<const Pack<S, EPT>*>(a + base);
    Pack<S, EPT> ib = *reinterpret_cast<const Pack<S, EPT>*>(b + base);
    Pack<S, EPT> ic = *reinterpret_cast<const Pack<S, EPT>*>(c + base);
    Pack<S, EPT> o0, o1;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      C r0, r1;
      Op::f(Io::in(ia.v[i]), Io::in(ib.v[i]), Io::in(ic.v[i]), r0, r1);
      o0.v[i] = Io::out(r0);
      o1.v[i] = Io::out(r1);
    }
    store_nt(o0, y0 + base);
    store_nt(o1, y1 + base);
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      if (base + i < n) {
        C r0, r1;
        Op::f(Io::in(a[base + i]), Io::in(b[base + i]), Io::in(c[base + i]), r0, r1);
        y0[base + i] = Io::out(r0);
        y1[base + i] = Io::out(r1);
      }
    }
  }
}

// elements per lane: 16 bytes of storage per lane and operand
template <class S>
constexpr int ept_for() { return 16 / (int)sizeof(S); }

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <class Io, class Op>
libm_hip_status launch_unary(const void* x, void* y, size_t n, void* stream, const char* name) {
  if (n == 0) return LIBM_HIP_OK;
  if (!x || !y) {
    set_error("libm_hip: NULL pointer with n > 0");
    return LIBM_HIP_ERR_INVALID;
  }
  typedef typename Io::S S;
  constexpr int EPT = ept_for<S>();
  size_t per_block = (size_t)BLOCK * EPT;
  size_t blocks = (n + per_block - 1) / per_block;
  if (blocks > 0x7fffffffull) {
    set_error("libm_hip: n too large for one launch");
    return LIBM_HIP_ERR_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  const S* xs = (const S*)x;
  S* ys = (S*)y;
  if (aligned16(x) && aligned16(y))
    hipLaunchKernelGGL((k_unary<Io, Op, EPT, true>), dim3((unsigned)blocks), dim3(BLOCK), 0, s, xs, ys, n);
  else
    hipLaunchKernelGGL((k_unary<Io, Op, EPT, false>), dim3((unsigned)blocks), dim3(BLOCK), 0, s, xs, ys, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    char buf[200];
    snprintf(buf, sizeof(buf), "libm_hip: %s launch failed: %s", name, hipGetErrorString(e));
    set_error(buf);
    return LIBM_HIP_ERR_HIP;
  }
  return LIBM_HIP_OK;
}

template <class Io, class Op>
libm_hip_status launch_binary(const void* a, const void* b, void* y, size_t n, void* stream,
                              const char* name) {
  if (n == 0) return LIBM_HIP_OK;
  if (!a || !b || !y) {
    set_error("libm_hip: NULL pointer with n > 0");
    return LIBM_HIP_ERR_INVALID;
  }
  typedef typename Io::S S;
  constexpr int EPT = ept_for<S>();
  size_t per_block = (size_t)BLOCK * EPT;
  size_t blocks = (n + per_block - 1) / per_block;
  if (blocks > 0x7fffffffull) {
    set_error("libm_hip: n too large for one launch");
    return LIBM_HIP_ERR_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  const S* as = (const S*)a;
  const S* bs = (const S*)b;
  S* ys = (S*)y;
  if (aligned16(a) && aligned16(b) && aligned16(y))
    hipLaunchKernelGGL((k_binary<Io, Op, EPT, true>), dim3((unsigned)blocks), dim3(BLOCK), 0, s, as, bs, ys, n);
  else
    hipLaunchKernelGGL((k_binary<Io, Op, EPT, false>), dim3((unsigned)blocks), dim3(BLOCK), 0, s, as, bs, ys, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    char buf[200];
    snprintf(buf, sizeof(buf), "libm_hip: %s launch failed: %s", name, hipGetErrorString(e));
    set_error(buf);
    return LIBM_HIP_ERR_HIP;
  }
  return LIBM_HIP_OK;
}

template <class Io, class Op>
libm_hip_status launch_ternary2(const void* a, const void* b, const void* c, void* y0, void* y1,
                                size_t n, void* stream, const char* name) {
  if (n == 0) return LIBM_HIP_OK;
  if (!a || !b || !c || !y0 || !y1) {
    set_error("libm_hip: NULL pointer with n > 0");
    return LIBM_HIP_ERR_INVALID;
  }
  typedef typename Io::S S;
  constexpr int EPT = ept_for<S>();
  size_t per_block = (size_t)BLOCK * EPT;
  size_t blocks = (n + per_block - 1) / per_block;
  if (blocks > 0x7fffffffull) {
    set_error("libm_hip: n too large for one launch");
    return LIBM_HIP_ERR_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  const S *as = (const S*)a, *bs = (const S*)b, *cs = (const S*)c;
  S *o0 = (S*)y0, *o1 = (S*)y1;
  if (aligned16(a) && aligned16(b) && aligned16(c) && aligned16(y0) && aligned16(y1))
    hipLaunchKernelGGL((k_ternary2<Io, Op, EPT, true>), dim3((unsigned)blocks), dim3(BLOCK), 0, s, as, bs, cs, o0, o1, n);
  else
    hipLaunchKernelGGL((k_ternary2<Io, Op, EPT, false>), dim3((unsigned)blocks), dim3(BLOCK), 0, s, as, bs, cs, o0, o1, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    char buf[200];
    snprintf(buf, sizeof(buf), "libm_hip: %s launch failed: %s", name, hipGetErrorString(e));
    set_error(buf);
    return LIBM_HIP_ERR_HIP;
  }
  return LIBM_HIP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* libm_hip_last_error(void) { return g_last_error; }
const char* libm_hip_version(void) { return "libm_hip 0.1 (gfx950)"; }

#define LMH_DEF_UNARY(fn, var, Op)                                                              \
  libm_hip_status libm_hip_##fn##_##var##_f64(const double* x, double* y, size_t n, void* s) { \
    return launch_unary<IoF64, Op>(x, y, n, s, #fn "_" #var "_f64");                           \
  }                                                                                             \
  libm_hip_status libm_hip_##fn##_##var##_f32(const float* x, float* y, size_t n, void* s) {   \
    return launch_unary<IoF32, Op>(x, y, n, s, #fn "_" #var "_f32");                           \
  }
#define LMH_DEF_UNARY_HALF(fn, Op)                                                                  \
  libm_hip_status libm_hip_##fn##_u10_bf16(const uint16_t* x, uint16_t* y, size_t n, void* s) {  \
    return launch_unary<IoBF16, Op>(x, y, n, s, #fn "_u10_bf16");                                \
  }                                                                                               \
  libm_hip_status libm_hip_##fn##_u10_f16(const uint16_t* x, uint16_t* y, size_t n, void* s) {   \
    return launch_unary<IoF16, Op>(x, y, n, s, #fn "_u10_f16");                                  \
  }                                                                                               \
  libm_hip_status libm_hip_##fn##_u10_f32_via_f64(const float* x, float* y, size_t n, void* s) { \
    return launch_unary<IoF32ViaF64, Op>(x, y, n, s, #fn "_u10_f32_via_f64");                    \
  }

LMH_DEF_UNARY(sin, u10, OpSinU10)
LMH_DEF_UNARY(sin, u35, OpSinU35)
LMH_DEF_UNARY(cos, u10, OpCosU10)
LMH_DEF_UNARY(cos, u35, OpCosU35)
LMH_DEF_UNARY(tan, u10, OpTanU10)
LMH_DEF_UNARY(tan, u35, OpTanU35)
LMH_DEF_UNARY(exp, u10, OpExpU10)
LMH_DEF_UNARY(exp2, u10, OpExp2U10)
LMH_DEF_UNARY(log, u10, OpLogU10)
LMH_DEF_UNARY(log2, u10, OpLog2U10)
LMH_DEF_UNARY(sinh, u10, OpSinhU10)
LMH_DEF_UNARY(cosh, u10, OpCoshU10)
LMH_DEF_UNARY(tanh, u10, OpTanhU10)
LMH_DEF_UNARY_HALF(sin, OpSinU10)
LMH_DEF_UNARY_HALF(cos, OpCosU10)
LMH_DEF_UNARY_HALF(tan, OpTanU10)
LMH_DEF_UNARY_HALF(exp, OpExpU10)
LMH_DEF_UNARY_HALF(exp2, OpExp2U10)
LMH_DEF_UNARY_HALF(log, OpLogU10)
LMH_DEF_UNARY_HALF(log2, OpLog2U10)
LMH_DEF_UNARY_HALF(sinh, OpSinhU10)
LMH_DEF_UNARY_HALF(cosh, OpCoshU10)
LMH_DEF_UNARY_HALF(tanh, OpTanhU10)

#define LMH_DEF_BINARY(fn, var, Io, T, tag, Op)                                                   \
  libm_hip_status libm_hip_##fn##var##_##tag(const T* a, const T* b, T* out, size_t n, void* s) { \
    return launch_binary<Io, Op>(a, b, out, n, s, #fn #var "_" #tag);                            \
  }

LMH_DEF_BINARY(pow, _u10, IoF64, double, f64, OpPowU10)
LMH_DEF_BINARY(pow, _u10, IoF32, float, f32, OpPowU10)
LMH_DEF_BINARY(pow, _u10, IoBF16, uint16_t, bf16, OpPowU10)
LMH_DEF_BINARY(pow, _u10, IoF16, uint16_t, f16, OpPowU10)
LMH_DEF_BINARY(pow, _u10, IoF32ViaF64, float, f32_via_f64, OpPowU10)
LMH_DEF_BINARY(atan2, _u10, IoF64, double, f64, OpAtan2U10)
LMH_DEF_BINARY(atan2, _u10, IoF32, float, f32, OpAtan2U10)
LMH_DEF_BINARY(atan2, _u10, IoBF16, uint16_t, bf16, OpAtan2U10)
LMH_DEF_BINARY(atan2, _u10, IoF16, uint16_t, f16, OpAtan2U10)
LMH_DEF_BINARY(atan2, _u10, IoF32ViaF64, float, f32_via_f64, OpAtan2U10)
LMH_DEF_BINARY(fmod, , IoF64, double, f64, OpFmod)
LMH_DEF_BINARY(fmod, , IoF32, float, f32, OpFmod)
LMH_DEF_BINARY(remainder, , IoF64, double, f64, OpRemainder)
LMH_DEF_BINARY(remainder, , IoF32, float, f32, OpRemainder)

}  // extern "C"

// ---------------------------------------------------------------------------
// backward entry points
// ---------------------------------------------------------------------------
extern "C" {
#define LMH_DEF_BWD(fn, Op)                                                                        \
  libm_hip_status libm_hip_##fn##_u10_f64_bwd(const double* x, const double* gy, double* gx,     \
                                               size_t n, void* s) {                                \
    return launch_binary<IoF64, Op>(x, gy, gx, n, s, #fn "_u10_f64_bwd");                          \
  }                                                                                                \
  libm_hip_status libm_hip_##fn##_u10_f32_bwd(const float* x, const float* gy, float* gx,        \
                                               size_t n, void* s) {                                \
    return launch_binary<IoF32, Op>(x, gy, gx, n, s, #fn "_u10_f32_bwd");                          \
  }
LMH_DEF_BWD(sin, OpSinBwd)
LMH_DEF_BWD(cos, OpCosBwd)
LMH_DEF_BWD(tan, OpTanBwd)
LMH_DEF_BWD(exp, OpExpBwd)
LMH_DEF_BWD(log, OpLogBwd)
LMH_DEF_BWD(tanh, OpTanhBwd)

libm_hip_status libm_hip_pow_u10_f64_bwd(const double* x, const double* y, const double* gout,
                                         double* gx, double* gy, size_t n, void* s) {
  return launch_ternary2<IoF64, OpPowBwd>(x, y, gout, gx, gy, n, s, "pow_u10_f64_bwd");
}
libm_hip_status libm_hip_pow_u10_f32_bwd(const float* x, const float* y, const float* gout,
                                         float* gx, float* gy, size_t n, void* s) {
  return launch_ternary2<IoF32, OpPowBwd>(x, y, gout, gx, gy, n, s, "pow_u10_f32_bwd");
}
libm_hip_status libm_hip_atan2_u10_f64_bwd(const double* y, const double* x, const double* gout,
                                           double* gy, double* gx, size_t n, void* s) {
  return launch_ternary2<IoF64, OpAtan2Bwd>(y, x, gout, gy, gx, n, s, "atan2_u10_f64_bwd");
}
libm_hip_status libm_hip_atan2_u10_f32_bwd(const float* y, const float* x, const float* gout,
                                           float* gy, float* gx, size_t n, void* s) {
  return launch_ternary2<IoF32, OpAtan2Bwd>(y, x, gout, gy, gx, n, s, "atan2_u10_f32_bwd");
}
}  // extern "C"

// ---------------------------------------------------------------------------
// generic dispatcher
// ---------------------------------------------------------------------------
namespace {
using namespace lmh_ops;

template <class Op>
libm_hip_status dispatch_unary(libm_hip_dtype t, const void* a, void* out, size_t n, void* s,
                               bool u35) {
  switch (t) {
    case LIBM_HIP_F64: return launch_unary<IoF64, Op>(a, out, n, s, "eval_f64");
    case LIBM_HIP_F32: return launch_unary<IoF32, Op>(a, out, n, s, "eval_f32");
    case LIBM_HIP_BF16: if (!u35) return launch_unary<IoBF16, Op>(a, out, n, s, "eval_bf16"); break;
    case LIBM_HIP_F16: if (!u35) return launch_unary<IoF16, Op>(a, out, n, s, "eval_f16"); break;
    case LIBM_HIP_F32_VIA_F64:
      if (!u35) return launch_unary<IoF32ViaF64, Op>(a, out, n, s, "eval_f32_via_f64");
      break;
  }
  set_error("libm_hip_eval: unsupported dtype for this function/variant");
  return LIBM_HIP_ERR_UNSUPPORTED;
}

template <class Op>
libm_hip_status dispatch_binary(libm_hip_dtype t, const void* a, const void* b, void* out,
                                size_t n, void* s, bool all_dtypes) {
  switch (t) {
    case LIBM_HIP_F64: return launch_binary<IoF64, Op>(a, b, out, n, s, "eval_f64");
    case LIBM_HIP_F32: return launch_binary<IoF32, Op>(a, b, out, n, s, "eval_f32");
    case LIBM_HIP_BF16:
      if (all_dtypes) return launch_binary<IoBF16, Op>(a, b, out, n, s, "eval_bf16");
      break;
    case LIBM_HIP_F16:
      if (all_dtypes) return launch_binary<IoF16, Op>(a, b, out, n, s, "eval_f16");
      break;
    case LIBM_HIP_F32_VIA_F64:
      if (all_dtypes) return launch_binary<IoF32ViaF64, Op>(a, b, out, n, s, "eval_f32_via_f64");
      break;
  }
  set_error("libm_hip_eval: unsupported dtype for this function");
  return LIBM_HIP_ERR_UNSUPPORTED;
}

}  // namespace

extern "C" libm_hip_status libm_hip_eval(libm_hip_fn fn, libm_hip_variant v, libm_hip_dtype t,
                                         const void* a, const void* b, void* out, size_t n,
                                         void* s) {
  bool u10 = v == LIBM_HIP_U10, u35 = v == LIBM_HIP_U35;
  switch (fn) {
    case LIBM_HIP_SIN:
      if (u10) return dispatch_unary<OpSinU10>(t, a, out, n, s, false);
      if (u35) return dispatch_unary<OpSinU35>(t, a, out, n, s, true);
      break;
    case LIBM_HIP_COS:
      if (u10) return dispatch_unary<OpCosU10>(t, a, out, n, s, false);
      if (u35) return dispatch_unary<OpCosU35>(t, a, out, n, s, true);
      break;
    case LIBM_HIP_TAN:
      if (u10) return dispatch_unary<OpTanU10>(t, a, out, n, s, false);
      if (u35) return dispatch_unary<OpTanU35>(t, a, out, n, s, true);
      break;
    case LIBM_HIP_EXP: if (u10) return dispatch_unary<OpExpU10>(t, a, out, n, s, false); break;
    case LIBM_HIP_EXP2: if (u10) return dispatch_unary<OpExp2U10>(t, a, out, n, s, false); break;
    case LIBM_HIP_LOG: if (u10) return dispatch_unary<OpLogU10>(t, a, out, n, s, false); break;
    case LIBM_HIP_LOG2: if (u10) return dispatch_unary<OpLog2U10>(t, a, out, n, s, false); break;
    case LIBM_HIP_SINH: if (u10) return dispatch_unary<OpSinhU10>(t, a, out, n, s, false); break;
    case LIBM_HIP_COSH: if (u10) return dispatch_unary<OpCoshU10>(t, a, out, n, s, false); break;
    case LIBM_HIP_TANH: if (u10) return dispatch_unary<OpTanhU10>(t, a, out, n, s, false); break;
    case LIBM_HIP_POW: if (u10) return dispatch_binary<OpPowU10>(t, a, b, out, n, s, true); break;
    case LIBM_HIP_ATAN2: if (u10) return dispatch_binary<OpAtan2U10>(t, a, b, out, n, s, true); break;
    case LIBM_HIP_FMOD:
      if (v == LIBM_HIP_EXACT) return dispatch_binary<OpFmod>(t, a, b, out, n, s, false);
      break;
    case LIBM_HIP_REMAINDER:
      if (v == LIBM_HIP_EXACT) return dispatch_binary<OpRemainder>(t, a, b, out, n, s, false);
      break;
    default: break;
  }
  set_error("libm_hip_eval: unsupported function/variant");
  return LIBM_HIP_ERR_UNSUPPORTED;
}
