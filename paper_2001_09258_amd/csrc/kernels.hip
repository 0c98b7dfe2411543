// The C ABI of libm_hip for the elementwise entry points: argument checks,
// launch shapes (default or autotuned), kernel launches (kernels.h), the
// generic dispatcher and the autotuner.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "abi_util.h"
#include "kernels.h"
#include "../../include/libm_hip.h"

namespace lmh_abi {
thread_local char g_last_error[256] = "";

void set_error(const char* msg) {
  strncpy(g_last_error, msg, sizeof(g_last_error) - 1);
  g_last_error[sizeof(g_last_error) - 1] = 0;
}
}  // namespace lmh_abi

namespace {
using namespace lmh_ops;
using namespace lmh_kernels;
using lmh_abi::set_error;

// ---------------------------------------------------------------------------
// launch configurations (autotuned)
// ---------------------------------------------------------------------------
// A launch is (workgroup size, packs per lane); a pack is 16 bytes of each
// operand.  The table holds the tuned choice per entry point and size bucket
// floor(log2 n); 0 means the default (256, 1).  Keys: (fn * 4 + variant) * 8
// + dtype, variant 3 = backward.
constexpr int NBUCKET = 48;
constexpr int NKEY = LIBM_HIP_NUM_FN * 4 * 8;
std::atomic<int> g_tune[NKEY][NBUCKET];
thread_local int g_force_cfg = 0;             // set only while tuning
std::once_flag g_tune_env_once;

struct Cfg {
  int block, packs;
};
inline int tune_key(int fn, int v, int t) { return (fn * 4 + v) * 8 + t; }
inline int nbucket(size_t n) {
  int b = 63 - __builtin_clzll((unsigned long long)n | 1ull);
  return b < NBUCKET ? b : NBUCKET - 1;
}
inline Cfg unpack_cfg(int v) { return v ? Cfg{v & 0xffff, v >> 16} : Cfg{256, 1}; }
int load_tune_file(const char* path);
inline Cfg pick_cfg(int key, size_t n) {
  std::call_once(g_tune_env_once, [] {
    const char* p = getenv("LIBM_HIP_TUNE_CACHE");
    if (p && *p) load_tune_file(p);
  });
  if (g_force_cfg) return unpack_cfg(g_force_cfg);
  if (key < 0 || key >= NKEY) return Cfg{256, 1};
  return unpack_cfg(g_tune[key][nbucket(n)].load(std::memory_order_relaxed));
}

int load_tune_file(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return -1;
  int key, b, blk, pk, count = 0;
  while (fscanf(f, "%d %d %d %d", &key, &b, &blk, &pk) == 4) {
    bool okb = blk == 64 || blk == 128 || blk == 256 || blk == 512 || blk == 1024;
    if (key >= 0 && key < NKEY && b >= 0 && b < NBUCKET && okb && (pk == 1 || pk == 2 || pk == 4)) {
      g_tune[key][b].store(blk | (pk << 16), std::memory_order_relaxed);
      ++count;
    }
  }
  fclose(f);
  return count;
}

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

inline libm_hip_status launch_error(const char* name) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    char buf[200];
    snprintf(buf, sizeof(buf), "libm_hip: %s launch failed: %s", name, hipGetErrorString(e));
    set_error(buf);
    return LIBM_HIP_ERR_HIP;
  }
  return LIBM_HIP_OK;
}

// grid for n elements, EPT per pack, cfg.packs packs per lane
inline bool grid_for(size_t n, int ept, Cfg c, unsigned& blocks) {
  size_t per_block = (size_t)c.block * c.packs * ept;
  size_t b = (n + per_block - 1) / per_block;
  if (b > 0x7fffffffull) {
    set_error("libm_hip: n too large for one launch");
    return false;
  }
  blocks = (unsigned)b;
  return true;
}

template <class Io, class OpF>
libm_hip_status launch_unary(const void* x, void* y, size_t n, void* stream, const char* name,
                             int key) {
  typedef typename EvalOp<Io, OpF>::type Op;
  if (n == 0) return LIBM_HIP_OK;
  if (!x || !y) {
    set_error("libm_hip: NULL pointer with n > 0");
    return LIBM_HIP_ERR_INVALID;
  }
  typedef typename Io::S S;
  constexpr int EPT = ept_for<S>();
  hipStream_t s = (hipStream_t)stream;
  const S* xs = (const S*)x;
  S* ys = (S*)y;
  bool vec = aligned16(x) && aligned16(y);
  unsigned blocks;
  if constexpr (Op::kSplit && sizeof(typename Io::C) == 8) {
    // binary64 evaluators: the per-wave gathering kernel, WPACKS packs per lane
    if (!grid_for(n, EPT, Cfg{BLOCK, WPACKS}, blocks)) return LIBM_HIP_ERR_INVALID;
    if (vec)
      hipLaunchKernelGGL((k_unary_wsplit<Io, Op, EPT, true>), dim3(blocks), dim3(BLOCK), 0, s, xs, ys, n);
    else
      hipLaunchKernelGGL((k_unary_wsplit<Io, Op, EPT, false>), dim3(blocks), dim3(BLOCK), 0, s, xs, ys, n);
  } else if constexpr (Op::kSplit) {
    // the workgroup-gathering kernel sizes its LDS queue to a 256-lane workgroup
    if (!grid_for(n, EPT, Cfg{BLOCK, 1}, blocks)) return LIBM_HIP_ERR_INVALID;
    if (vec)
      hipLaunchKernelGGL((k_unary_split<Io, Op, EPT, true>), dim3(blocks), dim3(BLOCK), 0, s, xs, ys, n);
    else
      hipLaunchKernelGGL((k_unary_split<Io, Op, EPT, false>), dim3(blocks), dim3(BLOCK), 0, s, xs, ys, n);
  } else {
    Cfg c = pick_cfg(key, n);
    if (!vec) c.packs = 1;
    if (!grid_for(n, EPT, c, blocks)) return LIBM_HIP_ERR_INVALID;
    dim3 g(blocks), b(c.block);
    if (!vec)
      hipLaunchKernelGGL((k_unary<Io, Op, EPT, false, 1>), g, b, 0, s, xs, ys, n);
    else if (c.packs == 4)
      hipLaunchKernelGGL((k_unary<Io, Op, EPT, true, 4>), g, b, 0, s, xs, ys, n);
    else if (c.packs == 2)
      hipLaunchKernelGGL((k_unary<Io, Op, EPT, true, 2>), g, b, 0, s, xs, ys, n);
    else
      hipLaunchKernelGGL((k_unary<Io, Op, EPT, true, 1>), g, b, 0, s, xs, ys, n);
  }
  return launch_error(name);
}

template <class Io, class OpF>
libm_hip_status launch_sincos(const void* x, void* ys, void* yc, size_t n, void* stream,
                              const char* name) {
  typedef typename EvalOp<Io, OpF>::type Op;
  if (n == 0) return LIBM_HIP_OK;
  if (!x || !ys || !yc) {
    set_error("libm_hip: NULL pointer with n > 0");
    return LIBM_HIP_ERR_INVALID;
  }
  typedef typename Io::S S;
  constexpr int EPT = ept_for<S>();
  hipStream_t s = (hipStream_t)stream;
  bool vec = aligned16(x) && aligned16(ys) && aligned16(yc);
  unsigned blocks;
  if (!grid_for(n, EPT, Cfg{BLOCK, 1}, blocks)) return LIBM_HIP_ERR_INVALID;
  const S* xs = (const S*)x;
  if (vec)
    hipLaunchKernelGGL((k_sincos_split<Io, Op, EPT, true>), dim3(blocks), dim3(BLOCK), 0, s, xs,
                       (S*)ys, (S*)yc, n);
  else
    hipLaunchKernelGGL((k_sincos_split<Io, Op, EPT, false>), dim3(blocks), dim3(BLOCK), 0, s, xs,
                       (S*)ys, (S*)yc, n);
  return launch_error(name);
}

template <class Io, class OpF>
libm_hip_status launch_binary(const void* a, const void* b, void* y, size_t n, void* stream,
                              const char* name, int key) {
  typedef typename EvalOp<Io, OpF>::type Op;
  if (n == 0) return LIBM_HIP_OK;
  if (!a || !b || !y) {
    set_error("libm_hip: NULL pointer with n > 0");
    return LIBM_HIP_ERR_INVALID;
  }
  typedef typename Io::S S;
  constexpr int EPT = ept_for<S>();
  Cfg c = pick_cfg(key, n);
  bool vec = aligned16(a) && aligned16(b) && aligned16(y);
  if (!vec) c.packs = 1;
  unsigned blocks;
  if (!grid_for(n, EPT, c, blocks)) return LIBM_HIP_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  const S* as = (const S*)a;
  const S* bs = (const S*)b;
  S* ys = (S*)y;
  dim3 g(blocks), bl(c.block);
  if (!vec)
    hipLaunchKernelGGL((k_binary<Io, Op, EPT, false, 1>), g, bl, 0, s, as, bs, ys, n);
  else if (c.packs == 4)
    hipLaunchKernelGGL((k_binary<Io, Op, EPT, true, 4>), g, bl, 0, s, as, bs, ys, n);
  else if (c.packs == 2)
    hipLaunchKernelGGL((k_binary<Io, Op, EPT, true, 2>), g, bl, 0, s, as, bs, ys, n);
  else
    hipLaunchKernelGGL((k_binary<Io, Op, EPT, true, 1>), g, bl, 0, s, as, bs, ys, n);
  return launch_error(name);
}

template <class Io, class Op>
libm_hip_status launch_ternary2(const void* a, const void* b, const void* c, void* y0, void* y1,
                                size_t n, void* stream, const char* name, int key) {
  if (n == 0) return LIBM_HIP_OK;
  if (!a || !b || !c || !y0 || !y1) {
    set_error("libm_hip: NULL pointer with n > 0");
    return LIBM_HIP_ERR_INVALID;
  }
  typedef typename Io::S S;
  constexpr int EPT = ept_for<S>();
  Cfg cf = pick_cfg(key, n);
  bool vec = aligned16(a) && aligned16(b) && aligned16(c) && aligned16(y0) && aligned16(y1);
  if (!vec) cf.packs = 1;
  unsigned blocks;
  if (!grid_for(n, EPT, cf, blocks)) return LIBM_HIP_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  const S *as = (const S*)a, *bs = (const S*)b, *cs = (const S*)c;
  S *o0 = (S*)y0, *o1 = (S*)y1;
  dim3 g(blocks), bl(cf.block);
  if (!vec)
    hipLaunchKernelGGL((k_ternary2<Io, Op, EPT, false, 1>), g, bl, 0, s, as, bs, cs, o0, o1, n);
  else if (cf.packs == 4)
    hipLaunchKernelGGL((k_ternary2<Io, Op, EPT, true, 4>), g, bl, 0, s, as, bs, cs, o0, o1, n);
  else if (cf.packs == 2)
    hipLaunchKernelGGL((k_ternary2<Io, Op, EPT, true, 2>), g, bl, 0, s, as, bs, cs, o0, o1, n);
  else
    hipLaunchKernelGGL((k_ternary2<Io, Op, EPT, true, 1>), g, bl, 0, s, as, bs, cs, o0, o1, n);
  return launch_error(name);
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* libm_hip_last_error(void) { return lmh_abi::g_last_error; }
const char* libm_hip_version(void) { return "libm_hip 0.1 (gfx950)"; }

#define LMH_KEY(FN, V, T) tune_key(LIBM_HIP_##FN, LIBM_HIP_##V, LIBM_HIP_##T)
#define LMH_DEF_UNARY(fn, var, Op, FN, V)                                                       \
  libm_hip_status libm_hip_##fn##_##var##_f64(const double* x, double* y, size_t n, void* s) { \
    return launch_unary<IoF64, Op>(x, y, n, s, #fn "_" #var "_f64", LMH_KEY(FN, V, F64));      \
  }                                                                                             \
  libm_hip_status libm_hip_##fn##_##var##_f32(const float* x, float* y, size_t n, void* s) {   \
    return launch_unary<IoF32, Op>(x, y, n, s, #fn "_" #var "_f32", LMH_KEY(FN, V, F32));      \
  }
#define LMH_DEF_UNARY_HALF(fn, Op, FN)                                                              \
  libm_hip_status libm_hip_##fn##_u10_bf16(const uint16_t* x, uint16_t* y, size_t n, void* s) {  \
    return launch_unary<IoBF16, Op>(x, y, n, s, #fn "_u10_bf16", LMH_KEY(FN, U10, BF16));        \
  }                                                                                               \
  libm_hip_status libm_hip_##fn##_u10_f16(const uint16_t* x, uint16_t* y, size_t n, void* s) {   \
    return launch_unary<IoF16, Op>(x, y, n, s, #fn "_u10_f16", LMH_KEY(FN, U10, F16));           \
  }                                                                                               \
  libm_hip_status libm_hip_##fn##_u10_f32_via_f64(const float* x, float* y, size_t n, void* s) { \
    return launch_unary<IoF32ViaF64, Op>(x, y, n, s, #fn "_u10_f32_via_f64",                     \
                                         LMH_KEY(FN, U10, F32_VIA_F64));                         \
  }

LMH_DEF_UNARY(sin, u10, OpSinU10, SIN, U10)
LMH_DEF_UNARY(sin, u35, OpSinU35, SIN, U35)
LMH_DEF_UNARY(cos, u10, OpCosU10, COS, U10)
LMH_DEF_UNARY(cos, u35, OpCosU35, COS, U35)
LMH_DEF_UNARY(tan, u10, OpTanU10, TAN, U10)
LMH_DEF_UNARY(tan, u35, OpTanU35, TAN, U35)
LMH_DEF_UNARY(exp, u10, OpExpU10, EXP, U10)
LMH_DEF_UNARY(exp2, u10, OpExp2U10, EXP2, U10)
LMH_DEF_UNARY(log, u10, OpLogU10, LOG, U10)
LMH_DEF_UNARY(log, u35, OpLogU35, LOG, U35)
LMH_DEF_UNARY(log2, u10, OpLog2U10, LOG2, U10)
LMH_DEF_UNARY(sinh, u10, OpSinhU10, SINH, U10)
LMH_DEF_UNARY(cosh, u10, OpCoshU10, COSH, U10)
LMH_DEF_UNARY(tanh, u10, OpTanhU10, TANH, U10)
LMH_DEF_UNARY(sinh, u35, OpSinhU35, SINH, U35)
LMH_DEF_UNARY(cosh, u35, OpCoshU35, COSH, U35)
LMH_DEF_UNARY(tanh, u35, OpTanhU35, TANH, U35)
LMH_DEF_UNARY(asin, u10, OpAsinU10, ASIN, U10)
LMH_DEF_UNARY(asin, u35, OpAsinU35, ASIN, U35)
LMH_DEF_UNARY(acos, u10, OpAcosU10, ACOS, U10)
LMH_DEF_UNARY(acos, u35, OpAcosU35, ACOS, U35)
LMH_DEF_UNARY(atan, u10, OpAtanU10, ATAN, U10)
LMH_DEF_UNARY(atan, u35, OpAtanU35, ATAN, U35)
LMH_DEF_UNARY(log10, u10, OpLog10U10, LOG10, U10)
LMH_DEF_UNARY(log1p, u10, OpLog1pU10, LOG1P, U10)
LMH_DEF_UNARY(exp10, u10, OpExp10U10, EXP10, U10)
LMH_DEF_UNARY(expm1, u10, OpExpm1U10, EXPM1, U10)
LMH_DEF_UNARY(cbrt, u10, OpCbrtU10, CBRT, U10)
LMH_DEF_UNARY(asinh, u10, OpAsinhU10, ASINH, U10)
LMH_DEF_UNARY(acosh, u10, OpAcoshU10, ACOSH, U10)
LMH_DEF_UNARY(atanh, u10, OpAtanhU10, ATANH, U10)
LMH_DEF_UNARY(erf, u10, OpErfU10, ERF, U10)
LMH_DEF_UNARY(erfc, u10, OpErfcU10, ERFC, U10)
LMH_DEF_UNARY(lgamma, u10, OpLgammaU10, LGAMMA, U10)
LMH_DEF_UNARY(tgamma, u10, OpTgammaU10, TGAMMA, U10)
LMH_DEF_UNARY_HALF(sin, OpSinU10, SIN)
LMH_DEF_UNARY_HALF(cos, OpCosU10, COS)
LMH_DEF_UNARY_HALF(tan, OpTanU10, TAN)
LMH_DEF_UNARY_HALF(exp, OpExpU10, EXP)
LMH_DEF_UNARY_HALF(exp2, OpExp2U10, EXP2)
LMH_DEF_UNARY_HALF(log, OpLogU10, LOG)
LMH_DEF_UNARY_HALF(log2, OpLog2U10, LOG2)
LMH_DEF_UNARY_HALF(sinh, OpSinhU10, SINH)
LMH_DEF_UNARY_HALF(cosh, OpCoshU10, COSH)
LMH_DEF_UNARY_HALF(tanh, OpTanhU10, TANH)
LMH_DEF_UNARY_HALF(asin, OpAsinU10, ASIN)
LMH_DEF_UNARY_HALF(acos, OpAcosU10, ACOS)
LMH_DEF_UNARY_HALF(atan, OpAtanU10, ATAN)
LMH_DEF_UNARY_HALF(log10, OpLog10U10, LOG10)
LMH_DEF_UNARY_HALF(log1p, OpLog1pU10, LOG1P)
LMH_DEF_UNARY_HALF(exp10, OpExp10U10, EXP10)
LMH_DEF_UNARY_HALF(expm1, OpExpm1U10, EXPM1)
LMH_DEF_UNARY_HALF(cbrt, OpCbrtU10, CBRT)
LMH_DEF_UNARY_HALF(asinh, OpAsinhU10, ASINH)
LMH_DEF_UNARY_HALF(acosh, OpAcoshU10, ACOSH)
LMH_DEF_UNARY_HALF(atanh, OpAtanhU10, ATANH)
LMH_DEF_UNARY_HALF(erf, OpErfU10, ERF)
LMH_DEF_UNARY_HALF(erfc, OpErfcU10, ERFC)
LMH_DEF_UNARY_HALF(lgamma, OpLgammaU10, LGAMMA)
LMH_DEF_UNARY_HALF(tgamma, OpTgammaU10, TGAMMA)

#define LMH_DEF_SINCOS(var, Io, T, tag, Op)                                                        \
  libm_hip_status libm_hip_sincos_##var##_##tag(const T* x, T* s, T* c, size_t n, void* stream) {  \
    return launch_sincos<Io, Op>(x, s, c, n, stream, "sincos_" #var "_" #tag);                      \
  }
LMH_DEF_SINCOS(u10, IoF64, double, f64, OpSinCosU10)
LMH_DEF_SINCOS(u10, IoF32, float, f32, OpSinCosU10)
LMH_DEF_SINCOS(u10, IoBF16, uint16_t, bf16, OpSinCosU10)
LMH_DEF_SINCOS(u10, IoF16, uint16_t, f16, OpSinCosU10)
LMH_DEF_SINCOS(u10, IoF32ViaF64, float, f32_via_f64, OpSinCosU10)
LMH_DEF_SINCOS(u35, IoF64, double, f64, OpSinCosU35)
LMH_DEF_SINCOS(u35, IoF32, float, f32, OpSinCosU35)

#define LMH_DEF_BINARY(fn, var, Io, T, tag, Op, KEY)                                              \
  libm_hip_status libm_hip_##fn##var##_##tag(const T* a, const T* b, T* out, size_t n, void* s) { \
    return launch_binary<Io, Op>(a, b, out, n, s, #fn #var "_" #tag, KEY);                       \
  }

LMH_DEF_BINARY(pow, _u10, IoF64, double, f64, OpPowU10, LMH_KEY(POW, U10, F64))
LMH_DEF_BINARY(pow, _u10, IoF32, float, f32, OpPowU10, LMH_KEY(POW, U10, F32))
LMH_DEF_BINARY(pow, _u10, IoBF16, uint16_t, bf16, OpPowU10, LMH_KEY(POW, U10, BF16))
LMH_DEF_BINARY(pow, _u10, IoF16, uint16_t, f16, OpPowU10, LMH_KEY(POW, U10, F16))
LMH_DEF_BINARY(pow, _u10, IoF32ViaF64, float, f32_via_f64, OpPowU10, LMH_KEY(POW, U10, F32_VIA_F64))
LMH_DEF_BINARY(atan2, _u10, IoF64, double, f64, OpAtan2U10, LMH_KEY(ATAN2, U10, F64))
LMH_DEF_BINARY(atan2, _u10, IoF32, float, f32, OpAtan2U10, LMH_KEY(ATAN2, U10, F32))
LMH_DEF_BINARY(atan2, _u10, IoBF16, uint16_t, bf16, OpAtan2U10, LMH_KEY(ATAN2, U10, BF16))
LMH_DEF_BINARY(atan2, _u10, IoF16, uint16_t, f16, OpAtan2U10, LMH_KEY(ATAN2, U10, F16))
LMH_DEF_BINARY(atan2, _u10, IoF32ViaF64, float, f32_via_f64, OpAtan2U10, LMH_KEY(ATAN2, U10, F32_VIA_F64))
LMH_DEF_BINARY(atan2, _u35, IoF64, double, f64, OpAtan2U35, LMH_KEY(ATAN2, U35, F64))
LMH_DEF_BINARY(pow, _u35, IoF64, double, f64, OpPowU35, LMH_KEY(POW, U35, F64))
LMH_DEF_BINARY(pow, _u35, IoF32, float, f32, OpPowU35, LMH_KEY(POW, U35, F32))
LMH_DEF_BINARY(atan2, _u35, IoF32, float, f32, OpAtan2U35, LMH_KEY(ATAN2, U35, F32))
LMH_DEF_BINARY(hypot, _u10, IoF64, double, f64, OpHypotU10, LMH_KEY(HYPOT, U10, F64))
LMH_DEF_BINARY(hypot, _u10, IoF32, float, f32, OpHypotU10, LMH_KEY(HYPOT, U10, F32))
LMH_DEF_BINARY(hypot, _u10, IoBF16, uint16_t, bf16, OpHypotU10, LMH_KEY(HYPOT, U10, BF16))
LMH_DEF_BINARY(hypot, _u10, IoF16, uint16_t, f16, OpHypotU10, LMH_KEY(HYPOT, U10, F16))
LMH_DEF_BINARY(hypot, _u10, IoF32ViaF64, float, f32_via_f64, OpHypotU10, LMH_KEY(HYPOT, U10, F32_VIA_F64))
LMH_DEF_BINARY(fmod, , IoF64, double, f64, OpFmod, LMH_KEY(FMOD, EXACT, F64))
LMH_DEF_BINARY(fmod, , IoF32, float, f32, OpFmod, LMH_KEY(FMOD, EXACT, F32))
LMH_DEF_BINARY(fdim, , IoF64, double, f64, OpFdim, LMH_KEY(FDIM, EXACT, F64))
LMH_DEF_BINARY(fdim, , IoF32, float, f32, OpFdim, LMH_KEY(FDIM, EXACT, F32))
LMH_DEF_BINARY(fmax, , IoF64, double, f64, OpFmax, LMH_KEY(FMAX, EXACT, F64))
LMH_DEF_BINARY(fmax, , IoF32, float, f32, OpFmax, LMH_KEY(FMAX, EXACT, F32))
LMH_DEF_BINARY(fmin, , IoF64, double, f64, OpFmin, LMH_KEY(FMIN, EXACT, F64))
LMH_DEF_BINARY(fmin, , IoF32, float, f32, OpFmin, LMH_KEY(FMIN, EXACT, F32))
LMH_DEF_BINARY(copysign, , IoF64, double, f64, OpCopysign, LMH_KEY(COPYSIGN, EXACT, F64))
LMH_DEF_BINARY(copysign, , IoF32, float, f32, OpCopysign, LMH_KEY(COPYSIGN, EXACT, F32))
LMH_DEF_BINARY(nextafter, , IoF64, double, f64, OpNextafter, LMH_KEY(NEXTAFTER, EXACT, F64))
LMH_DEF_BINARY(nextafter, , IoF32, float, f32, OpNextafter, LMH_KEY(NEXTAFTER, EXACT, F32))

#define LMH_DEF_EXACT1(fn, Op, FN)                                                               \
  libm_hip_status libm_hip_##fn##_f64(const double* x, double* y, size_t n, void* s) {          \
    return launch_unary<IoF64, Op>(x, y, n, s, #fn "_f64", LMH_KEY(FN, EXACT, F64));             \
  }                                                                                              \
  libm_hip_status libm_hip_##fn##_f32(const float* x, float* y, size_t n, void* s) {            \
    return launch_unary<IoF32, Op>(x, y, n, s, #fn "_f32", LMH_KEY(FN, EXACT, F32));             \
  }
LMH_DEF_EXACT1(sqrt, OpSqrt, SQRT)
LMH_DEF_EXACT1(trunc, OpTrunc, TRUNC)
LMH_DEF_EXACT1(floor, OpFloor, FLOOR)
LMH_DEF_EXACT1(ceil, OpCeil, CEIL)
LMH_DEF_EXACT1(round, OpRound, ROUND)
LMH_DEF_EXACT1(rint, OpRint, RINT)
LMH_DEF_EXACT1(fabs, OpFabs, FABS)
LMH_DEF_EXACT1(logb, OpLogb, LOGB)
LMH_DEF_BINARY(remainder, , IoF64, double, f64, OpRemainder, LMH_KEY(REMAINDER, EXACT, F64))
LMH_DEF_BINARY(remainder, , IoF32, float, f32, OpRemainder, LMH_KEY(REMAINDER, EXACT, F32))

}  // extern "C"

// ---------------------------------------------------------------------------
// backward entry points
// ---------------------------------------------------------------------------
extern "C" {
#define LMH_DEF_BWD(fn, Op, FN)                                                                      \
  libm_hip_status libm_hip_##fn##_u10_f64_bwd(const double* x, const double* gy, double* gx,     \
                                               size_t n, void* s) {                                \
    return launch_binary<IoF64, Op>(x, gy, gx, n, s, #fn "_u10_f64_bwd", tune_key(FN, 3, 0));      \
  }                                                                                                \
  libm_hip_status libm_hip_##fn##_u10_f32_bwd(const float* x, const float* gy, float* gx,        \
                                               size_t n, void* s) {                                \
    return launch_binary<IoF32, Op>(x, gy, gx, n, s, #fn "_u10_f32_bwd", tune_key(FN, 3, 1));      \
  }
LMH_DEF_BWD(sin, OpSinBwd, LIBM_HIP_SIN)
LMH_DEF_BWD(cos, OpCosBwd, LIBM_HIP_COS)
LMH_DEF_BWD(tan, OpTanBwd, LIBM_HIP_TAN)
LMH_DEF_BWD(exp, OpExpBwd, LIBM_HIP_EXP)
LMH_DEF_BWD(log, OpLogBwd, LIBM_HIP_LOG)
LMH_DEF_BWD(tanh, OpTanhBwd, LIBM_HIP_TANH)

libm_hip_status libm_hip_pow_u10_f64_bwd(const double* x, const double* y, const double* gout,
                                         double* gx, double* gy, size_t n, void* s) {
  return launch_ternary2<IoF64, OpPowBwd>(x, y, gout, gx, gy, n, s, "pow_u10_f64_bwd",
                                          tune_key(LIBM_HIP_POW, 3, 0));
}
libm_hip_status libm_hip_pow_u10_f32_bwd(const float* x, const float* y, const float* gout,
                                         float* gx, float* gy, size_t n, void* s) {
  return launch_ternary2<IoF32, OpPowBwd>(x, y, gout, gx, gy, n, s, "pow_u10_f32_bwd",
                                          tune_key(LIBM_HIP_POW, 3, 1));
}
libm_hip_status libm_hip_atan2_u10_f64_bwd(const double* y, const double* x, const double* gout,
                                           double* gy, double* gx, size_t n, void* s) {
  return launch_ternary2<IoF64, OpAtan2Bwd>(y, x, gout, gy, gx, n, s, "atan2_u10_f64_bwd",
                                            tune_key(LIBM_HIP_ATAN2, 3, 0));
}
libm_hip_status libm_hip_atan2_u10_f32_bwd(const float* y, const float* x, const float* gout,
                                           float* gy, float* gx, size_t n, void* s) {
  return launch_ternary2<IoF32, OpAtan2Bwd>(y, x, gout, gy, gx, n, s, "atan2_u10_f32_bwd",
                                            tune_key(LIBM_HIP_ATAN2, 3, 1));
}
}  // extern "C"

// ---------------------------------------------------------------------------
// generic dispatcher
// ---------------------------------------------------------------------------
namespace {
using namespace lmh_ops;

template <class Op>
libm_hip_status dispatch_unary(libm_hip_dtype t, const void* a, void* out, size_t n, void* s,
                               bool u35, int key) {
  switch (t) {
    case LIBM_HIP_F64: return launch_unary<IoF64, Op>(a, out, n, s, "eval_f64", key);
    case LIBM_HIP_F32: return launch_unary<IoF32, Op>(a, out, n, s, "eval_f32", key);
    case LIBM_HIP_BF16: if (!u35) return launch_unary<IoBF16, Op>(a, out, n, s, "eval_bf16", key); break;
    case LIBM_HIP_F16: if (!u35) return launch_unary<IoF16, Op>(a, out, n, s, "eval_f16", key); break;
    case LIBM_HIP_F32_VIA_F64:
      if (!u35) return launch_unary<IoF32ViaF64, Op>(a, out, n, s, "eval_f32_via_f64", key);
      break;
  }
  set_error("libm_hip_eval: unsupported dtype for this function/variant");
  return LIBM_HIP_ERR_UNSUPPORTED;
}

template <class Op>
libm_hip_status dispatch_binary(libm_hip_dtype t, const void* a, const void* b, void* out,
                                size_t n, void* s, bool all_dtypes, int key) {
  switch (t) {
    case LIBM_HIP_F64: return launch_binary<IoF64, Op>(a, b, out, n, s, "eval_f64", key);
    case LIBM_HIP_F32: return launch_binary<IoF32, Op>(a, b, out, n, s, "eval_f32", key);
    case LIBM_HIP_BF16:
      if (all_dtypes) return launch_binary<IoBF16, Op>(a, b, out, n, s, "eval_bf16", key);
      break;
    case LIBM_HIP_F16:
      if (all_dtypes) return launch_binary<IoF16, Op>(a, b, out, n, s, "eval_f16", key);
      break;
    case LIBM_HIP_F32_VIA_F64:
      if (all_dtypes) return launch_binary<IoF32ViaF64, Op>(a, b, out, n, s, "eval_f32_via_f64", key);
      break;
  }
  set_error("libm_hip_eval: unsupported dtype for this function");
  return LIBM_HIP_ERR_UNSUPPORTED;
}

}  // namespace

// ---------------------------------------------------------------------------
// integer-operand functions: ldexp, ilogb, frexp (binary64, binary32)
// ---------------------------------------------------------------------------
namespace {
inline unsigned map_grid(size_t n) {
  size_t b = (n + MAP_BLOCK - 1) / MAP_BLOCK;
  return (unsigned)(b < 65536 ? b : 65536);
}
template <class T>
libm_hip_status run_ldexp(const T* x, const int32_t* e, T* y, size_t n, void* s, const char* nm) {
  if (n == 0) return LIBM_HIP_OK;
  if (!x || !e || !y) {
    set_error("libm_hip: NULL pointer with n > 0");
    return LIBM_HIP_ERR_INVALID;
  }
  hipLaunchKernelGGL((k_ldexp<T, OpIntFns>), dim3(map_grid(n)), dim3(MAP_BLOCK), 0,
                     (hipStream_t)s, x, (const int*)e, y, n);
  return launch_error(nm);
}
template <class T>
libm_hip_status run_ilogb(const T* x, int32_t* e, size_t n, void* s, const char* nm) {
  if (n == 0) return LIBM_HIP_OK;
  if (!x || !e) {
    set_error("libm_hip: NULL pointer with n > 0");
    return LIBM_HIP_ERR_INVALID;
  }
  hipLaunchKernelGGL((k_ilogb<T, OpIntFns>), dim3(map_grid(n)), dim3(MAP_BLOCK), 0,
                     (hipStream_t)s, x, (int*)e, n);
  return launch_error(nm);
}
template <class T>
libm_hip_status run_frexp(const T* x, T* m, int32_t* e, size_t n, void* s, const char* nm) {
  if (n == 0) return LIBM_HIP_OK;
  if (!x || !m || !e) {
    set_error("libm_hip: NULL pointer with n > 0");
    return LIBM_HIP_ERR_INVALID;
  }
  hipLaunchKernelGGL((k_frexp<T, OpIntFns>), dim3(map_grid(n)), dim3(MAP_BLOCK), 0,
                     (hipStream_t)s, x, m, (int*)e, n);
  return launch_error(nm);
}
#define LMH_MAP_CHECK(...)                                                                  \
  if (n == 0) return LIBM_HIP_OK;                                                           \
  if (__VA_ARGS__) {                                                                        \
    set_error("libm_hip: NULL pointer with n > 0");                                         \
    return LIBM_HIP_ERR_INVALID;                                                            \
  }
template <class T>
libm_hip_status run_modf(const T* x, T* f, T* ip, size_t n, void* s, const char* nm) {
  LMH_MAP_CHECK(!x || !f || !ip)
  hipLaunchKernelGGL((k_modf<T, OpIntFns>), dim3(map_grid(n)), dim3(MAP_BLOCK), 0,
                     (hipStream_t)s, x, f, ip, n);
  return launch_error(nm);
}
template <class T>
libm_hip_status run_fma(const T* a, const T* b, const T* c, T* y, size_t n, void* s,
                        const char* nm) {
  LMH_MAP_CHECK(!a || !b || !c || !y)
  hipLaunchKernelGGL((k_fma<T, OpIntFns>), dim3(map_grid(n)), dim3(MAP_BLOCK), 0,
                     (hipStream_t)s, a, b, c, y, n);
  return launch_error(nm);
}
template <class T, bool ROUND>
libm_hip_status run_lrint(const T* x, int64_t* y, size_t n, void* s, const char* nm) {
  LMH_MAP_CHECK(!x || !y)
  hipLaunchKernelGGL((k_lrint<T, OpIntFns, ROUND>), dim3(map_grid(n)), dim3(MAP_BLOCK), 0,
                     (hipStream_t)s, x, (long long*)y, n);
  return launch_error(nm);
}
template <class T>
libm_hip_status run_remquo(const T* x, const T* y, T* r, int32_t* q, size_t n, void* s,
                           const char* nm) {
  LMH_MAP_CHECK(!x || !y || !r || !q)
  hipLaunchKernelGGL((k_remquo<T, OpIntFns>), dim3(map_grid(n)), dim3(MAP_BLOCK), 0,
                     (hipStream_t)s, x, y, r, (int*)q, n);
  return launch_error(nm);
}
#undef LMH_MAP_CHECK
}  // namespace

extern "C" {
#define LMH_DEF_MAPS(T, tag)                                                                     \
  libm_hip_status libm_hip_modf_##tag(const T* x, T* f, T* ip, size_t n, void* s) {            \
    return run_modf(x, f, ip, n, s, "modf_" #tag);                                              \
  }                                                                                              \
  libm_hip_status libm_hip_fma_##tag(const T* a, const T* b, const T* c, T* y, size_t n,       \
                                     void* s) {                                                  \
    return run_fma(a, b, c, y, n, s, "fma_" #tag);                                              \
  }                                                                                              \
  libm_hip_status libm_hip_lrint_##tag(const T* x, int64_t* y, size_t n, void* s) {            \
    return run_lrint<T, false>(x, y, n, s, "lrint_" #tag);                                      \
  }                                                                                              \
  libm_hip_status libm_hip_lround_##tag(const T* x, int64_t* y, size_t n, void* s) {           \
    return run_lrint<T, true>(x, y, n, s, "lround_" #tag);                                      \
  }                                                                                              \
  libm_hip_status libm_hip_remquo_##tag(const T* x, const T* y, T* r, int32_t* q, size_t n,    \
                                        void* s) {                                               \
    return run_remquo(x, y, r, q, n, s, "remquo_" #tag);                                        \
  }
LMH_DEF_MAPS(double, f64)
LMH_DEF_MAPS(float, f32)
#undef LMH_DEF_MAPS
libm_hip_status libm_hip_ldexp_f64(const double* x, const int32_t* e, double* y, size_t n, void* s) {
  return run_ldexp(x, e, y, n, s, "ldexp_f64");
}
libm_hip_status libm_hip_ldexp_f32(const float* x, const int32_t* e, float* y, size_t n, void* s) {
  return run_ldexp(x, e, y, n, s, "ldexp_f32");
}
libm_hip_status libm_hip_ilogb_f64(const double* x, int32_t* e, size_t n, void* s) {
  return run_ilogb(x, e, n, s, "ilogb_f64");
}
libm_hip_status libm_hip_ilogb_f32(const float* x, int32_t* e, size_t n, void* s) {
  return run_ilogb(x, e, n, s, "ilogb_f32");
}
libm_hip_status libm_hip_frexp_f64(const double* x, double* m, int32_t* e, size_t n, void* s) {
  return run_frexp(x, m, e, n, s, "frexp_f64");
}
libm_hip_status libm_hip_frexp_f32(const float* x, float* m, int32_t* e, size_t n, void* s) {
  return run_frexp(x, m, e, n, s, "frexp_f32");
}
}  // extern "C"

extern "C" libm_hip_status libm_hip_eval(libm_hip_fn fn, libm_hip_variant v, libm_hip_dtype t,
                                         const void* a, const void* b, void* out, size_t n,
                                         void* s) {
  bool u10 = v == LIBM_HIP_U10, u35 = v == LIBM_HIP_U35;
  const int key = tune_key(fn, v, t);
  switch (fn) {
    case LIBM_HIP_SIN:
      if (u10) return dispatch_unary<OpSinU10>(t, a, out, n, s, false, key);
      if (u35) return dispatch_unary<OpSinU35>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_COS:
      if (u10) return dispatch_unary<OpCosU10>(t, a, out, n, s, false, key);
      if (u35) return dispatch_unary<OpCosU35>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_TAN:
      if (u10) return dispatch_unary<OpTanU10>(t, a, out, n, s, false, key);
      if (u35) return dispatch_unary<OpTanU35>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_EXP: if (u10) return dispatch_unary<OpExpU10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_EXP2: if (u10) return dispatch_unary<OpExp2U10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_LOG:
      if (u10) return dispatch_unary<OpLogU10>(t, a, out, n, s, false, key);
      if (u35) return dispatch_unary<OpLogU35>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_LOG2: if (u10) return dispatch_unary<OpLog2U10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_SINH:
      if (u10) return dispatch_unary<OpSinhU10>(t, a, out, n, s, false, key);
      if (u35) return dispatch_unary<OpSinhU35>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_COSH:
      if (u10) return dispatch_unary<OpCoshU10>(t, a, out, n, s, false, key);
      if (u35) return dispatch_unary<OpCoshU35>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_TANH:
      if (u10) return dispatch_unary<OpTanhU10>(t, a, out, n, s, false, key);
      if (u35) return dispatch_unary<OpTanhU35>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_ASIN:
      if (u10) return dispatch_unary<OpAsinU10>(t, a, out, n, s, false, key);
      if (u35) return dispatch_unary<OpAsinU35>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_ACOS:
      if (u10) return dispatch_unary<OpAcosU10>(t, a, out, n, s, false, key);
      if (u35) return dispatch_unary<OpAcosU35>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_ATAN:
      if (u10) return dispatch_unary<OpAtanU10>(t, a, out, n, s, false, key);
      if (u35) return dispatch_unary<OpAtanU35>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_LOG10: if (u10) return dispatch_unary<OpLog10U10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_LOG1P: if (u10) return dispatch_unary<OpLog1pU10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_EXP10: if (u10) return dispatch_unary<OpExp10U10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_EXPM1: if (u10) return dispatch_unary<OpExpm1U10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_CBRT: if (u10) return dispatch_unary<OpCbrtU10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_ASINH: if (u10) return dispatch_unary<OpAsinhU10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_ACOSH: if (u10) return dispatch_unary<OpAcoshU10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_ATANH: if (u10) return dispatch_unary<OpAtanhU10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_ERF: if (u10) return dispatch_unary<OpErfU10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_LGAMMA: if (u10) return dispatch_unary<OpLgammaU10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_TGAMMA: if (u10) return dispatch_unary<OpTgammaU10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_ERFC: if (u10) return dispatch_unary<OpErfcU10>(t, a, out, n, s, false, key); break;
    case LIBM_HIP_HYPOT: if (u10) return dispatch_binary<OpHypotU10>(t, a, b, out, n, s, true, key); break;
    case LIBM_HIP_POW:
      if (u10) return dispatch_binary<OpPowU10>(t, a, b, out, n, s, true, key);
      if (u35) return dispatch_binary<OpPowU35>(t, a, b, out, n, s, false, key);
      break;
    case LIBM_HIP_ATAN2:
      if (u10) return dispatch_binary<OpAtan2U10>(t, a, b, out, n, s, true, key);
      if (u35) return dispatch_binary<OpAtan2U35>(t, a, b, out, n, s, false, key);
      break;
    case LIBM_HIP_FMOD:
      if (v == LIBM_HIP_EXACT) return dispatch_binary<OpFmod>(t, a, b, out, n, s, false, key);
      break;
    case LIBM_HIP_REMAINDER:
      if (v == LIBM_HIP_EXACT) return dispatch_binary<OpRemainder>(t, a, b, out, n, s, false, key);
      break;
    case LIBM_HIP_FDIM:
      if (v == LIBM_HIP_EXACT) return dispatch_binary<OpFdim>(t, a, b, out, n, s, false, key);
      break;
    case LIBM_HIP_FMAX:
      if (v == LIBM_HIP_EXACT) return dispatch_binary<OpFmax>(t, a, b, out, n, s, false, key);
      break;
    case LIBM_HIP_FMIN:
      if (v == LIBM_HIP_EXACT) return dispatch_binary<OpFmin>(t, a, b, out, n, s, false, key);
      break;
    case LIBM_HIP_SQRT:
      if (v == LIBM_HIP_EXACT) return dispatch_unary<OpSqrt>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_TRUNC:
      if (v == LIBM_HIP_EXACT) return dispatch_unary<OpTrunc>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_FLOOR:
      if (v == LIBM_HIP_EXACT) return dispatch_unary<OpFloor>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_CEIL:
      if (v == LIBM_HIP_EXACT) return dispatch_unary<OpCeil>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_ROUND:
      if (v == LIBM_HIP_EXACT) return dispatch_unary<OpRound>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_RINT:
      if (v == LIBM_HIP_EXACT) return dispatch_unary<OpRint>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_FABS:
      if (v == LIBM_HIP_EXACT) return dispatch_unary<OpFabs>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_LOGB:
      if (v == LIBM_HIP_EXACT) return dispatch_unary<OpLogb>(t, a, out, n, s, true, key);
      break;
    case LIBM_HIP_COPYSIGN:
      if (v == LIBM_HIP_EXACT) return dispatch_binary<OpCopysign>(t, a, b, out, n, s, false, key);
      break;
    case LIBM_HIP_NEXTAFTER:
      if (v == LIBM_HIP_EXACT) return dispatch_binary<OpNextafter>(t, a, b, out, n, s, false, key);
      break;
    default: break;
  }
  set_error("libm_hip_eval: unsupported function/variant");
  return LIBM_HIP_ERR_UNSUPPORTED;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
extern "C" libm_hip_status libm_hip_tune(libm_hip_fn fn, libm_hip_variant v, libm_hip_dtype t,
                                         const void* a, const void* b, void* out, size_t n,
                                         void* stream, int* best_block, int* best_packs) {
  static const int blocks[] = {64, 128, 256, 512, 1024};
  static const int packs[] = {1, 2, 4};
  if (n == 0 || !a || !out) {
    set_error("libm_hip_tune: needs n > 0 and valid buffers");
    return LIBM_HIP_ERR_INVALID;
  }
  if ((int)fn < 0 || fn >= LIBM_HIP_NUM_FN || (int)v < 0 || v > LIBM_HIP_EXACT || (int)t < 0 ||
      t > LIBM_HIP_F32_VIA_F64) {
    set_error("libm_hip_tune: unknown function, variant or dtype");
    return LIBM_HIP_ERR_UNSUPPORTED;
  }
  if (fn == LIBM_HIP_SIN || fn == LIBM_HIP_COS || fn == LIBM_HIP_TAN) {
    // the gathering trig kernels have one shape (their LDS queue is sized
    // for a 256-lane workgroup)
    if (best_block) *best_block = BLOCK;
    if (best_packs) *best_packs = 1;
    return LIBM_HIP_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("libm_hip_tune: event creation failed");
    return LIBM_HIP_ERR_HIP;
  }
  // every shape: one warm-up launch, then the fastest of three rounds of
  // three launches.  The default shape is timed first and is replaced only
  // by a shape at least 2% faster, so timing noise does not pick shapes.
  const int def = 256 | (1 << 16);
  float def_ms = 1e30f, best_ms = 1e30f;
  int best = 0;
  libm_hip_status st = LIBM_HIP_OK;
  hipError_t he = hipSuccess;
  for (int ci = -1; ci < 15 && st == LIBM_HIP_OK && he == hipSuccess; ++ci) {
    int cfg = ci < 0 ? def : (blocks[ci / 3] | (packs[ci % 3] << 16));
    if (ci >= 0 && cfg == def) continue;
    g_force_cfg = cfg;
    st = libm_hip_eval(fn, v, t, a, b, out, n, stream);          // warm-up
    float ms_cfg = 1e30f;
    for (int round = 0; round < 3 && st == LIBM_HIP_OK && he == hipSuccess; ++round) {
      he = hipEventRecord(e0, s);
      for (int r = 0; r < 3 && st == LIBM_HIP_OK; ++r)
        st = libm_hip_eval(fn, v, t, a, b, out, n, stream);
      if (he == hipSuccess) he = hipEventRecord(e1, s);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he == hipSuccess && ms < ms_cfg) ms_cfg = ms;
    }
    if (st != LIBM_HIP_OK || he != hipSuccess) break;
    if (ci < 0) {
      def_ms = ms_cfg;
    } else if (ms_cfg < best_ms) {
      best_ms = ms_cfg;
      best = cfg;
    }
  }
  if (!(best_ms < 0.98f * def_ms)) best = 0;                   // keep the default
  g_force_cfg = 0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LIBM_HIP_OK) return st;
  if (he != hipSuccess) {
    set_error(hipGetErrorString(he));
    return LIBM_HIP_ERR_HIP;
  }
  g_tune[tune_key(fn, v, t)][nbucket(n)].store(best, std::memory_order_relaxed);
  Cfg c = unpack_cfg(best);
  if (best_block) *best_block = c.block;
  if (best_packs) *best_packs = c.packs;
  return LIBM_HIP_OK;
}

extern "C" libm_hip_status libm_hip_tune_save(const char* path) {
  FILE* f = path ? fopen(path, "w") : nullptr;
  if (!f) {
    set_error("libm_hip_tune_save: cannot open file");
    return LIBM_HIP_ERR_INVALID;
  }
  for (int k = 0; k < NKEY; ++k)
    for (int b = 0; b < NBUCKET; ++b) {
      int v = g_tune[k][b].load(std::memory_order_relaxed);
      if (v) fprintf(f, "%d %d %d %d\n", k, b, v & 0xffff, v >> 16);
    }
  fclose(f);
  return LIBM_HIP_OK;
}

extern "C" libm_hip_status libm_hip_tune_load(const char* path) {
  if (!path || load_tune_file(path) < 0) {
    set_error("libm_hip_tune_load: cannot read file");
    return LIBM_HIP_ERR_INVALID;
  }
  return LIBM_HIP_OK;
}

extern "C" void libm_hip_tune_reset(void) {
  for (int k = 0; k < NKEY; ++k)
    for (int b = 0; b < NBUCKET; ++b) g_tune[k][b].store(0, std::memory_order_relaxed);
}
