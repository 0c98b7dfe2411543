#include <hip/hip_runtime.h>
// Probe kernels for counting the vector ALU work of each evaluator piece
// (compiled to gfx950 assembly by count_ops.py, never linked into the
// library).  Each kernel runs exactly one path of one evaluator on one
// element per lane.
#include "../csrc/eval_f64.h"
#include "../csrc/eval_f32.h"
using namespace lmh;
#define K1(NAME, T, EXPR) __global__ void NAME(const T* x, T* y) { int i = threadIdx.x; T v = x[i]; y[i] = (EXPR); }
#define KS(NAME, T, EXPR) __global__ void NAME(const T* x, T* y) { int i = threadIdx.x; T v = x[i]; auto s = (EXPR); y[i] = s.r.hi + s.r.lo + s.j; }
// binary64 pieces
KS(p64_sincw, double, sincos_fast(v, false))
KS(p64_coscw, double, sincos_fast(v, true))
KS(p64_tancw, double, tan_fast(v))
KS(p64_sinph, double, sincos_slow(v, false))
KS(p64_cosph, double, sincos_slow(v, true))
KS(p64_tanph, double, tan_slow(v))
__global__ void p64_sinfin(const double* x, double* y) { int i = threadIdx.x; Trig64 s{mk(x[i], x[i+64]), x[i+128]}; y[i] = sin_finish_u10(x[i+192], s); }
__global__ void p64_sinfin35(const double* x, double* y) { int i = threadIdx.x; Trig64 s{mk(x[i], x[i+64]), x[i+128]}; y[i] = sin_finish_u35(x[i+192], s); }
__global__ void p64_tanfin(const double* x, double* y) { int i = threadIdx.x; Trig64 s{mk(x[i], x[i+64]), x[i+128]}; y[i] = tan_finish_u10(x[i+192], s); }
__global__ void p64_tanfin35(const double* x, double* y) { int i = threadIdx.x; Trig64 s{mk(x[i], x[i+64]), x[i+128]}; y[i] = tan_finish_u35(x[i+192], s); }
K1(p64_exp, double, exp_u10(v))
K1(p64_exp2, double, exp2_u10(v))
K1(p64_log, double, log_u10(v))
K1(p64_log2, double, log2_u10(v))
K1(p64_sinh, double, sinh_u10(v))
K1(p64_cosh, double, cosh_u10(v))
K1(p64_tanh, double, tanh_u10(v))
K1(p64_log35, double, log_u35(v))
K1(p64_asin, double, asin_u10(v))
K1(p64_asin35, double, asin_u35(v))
K1(p64_acos, double, acos_u10(v))
K1(p64_acos35, double, acos_u35(v))
K1(p64_atan, double, atan_u10(v))
K1(p64_atan35, double, atan_u35(v))
__global__ void p64_pow(const double* x, double* y) { int i = threadIdx.x; y[i] = pow_u10(x[i], x[i+64]); }
__global__ void p64_atan2(const double* x, double* y) { int i = threadIdx.x; y[i] = atan2_u10(x[i], x[i+64]); }
__global__ void p64_hypot(const double* x, double* y) { int i = threadIdx.x; y[i] = hypot_u10(x[i], x[i+64]); }
__global__ void p64_atan235(const double* x, double* y) { int i = threadIdx.x; y[i] = atan2_u35(x[i], x[i+64]); }
__global__ void p64_pow35(const double* x, double* y) { int i = threadIdx.x; y[i] = pow_u35(x[i], x[i+64]); }
K1(p64_sinh35, double, sinh_u35(v))
K1(p64_cosh35, double, cosh_u35(v))
K1(p64_tanh35, double, tanh_u35(v))
K1(p64_log10, double, log10_u10(v))
K1(p64_log1p, double, log1p_u10(v))
K1(p64_exp10, double, exp10_u10(v))
K1(p64_expm1, double, expm1_u10(v))
K1(p64_cbrt, double, cbrt_u10(v))
K1(p64_asinh, double, asinh_u10(v))
K1(p64_acosh, double, acosh_u10(v))
K1(p64_atanh, double, atanh_u10(v))
K1(p64_erf, double, erf_u10(v))
K1(p64_erfc, double, erfc_u10(v))
// binary32 pieces
KS(p32_sincw, float, sincosf_fast(v, false))
KS(p32_coscw, float, sincosf_fast(v, true))
KS(p32_tancw, float, tanf_fast(v))
KS(p32_sinph, float, sincosf_slow(v, false))
KS(p32_cosph, float, sincosf_slow(v, true))
KS(p32_tanph, float, tanf_slow(v))
__global__ void p32_sinfin(const float* x, float* y) { int i = threadIdx.x; Trig32 s{mk(x[i], x[i+64]), x[i+128]}; y[i] = sinf_finish_u10(x[i+192], s); }
__global__ void p32_sinfin35(const float* x, float* y) { int i = threadIdx.x; Trig32 s{mk(x[i], x[i+64]), x[i+128]}; y[i] = sinf_finish_u35(x[i+192], s); }
__global__ void p32_tanfin(const float* x, float* y) { int i = threadIdx.x; Trig32 s{mk(x[i], x[i+64]), x[i+128]}; y[i] = tanf_finish_u10(x[i+192], s); }
__global__ void p32_tanfin35(const float* x, float* y) { int i = threadIdx.x; Trig32 s{mk(x[i], x[i+64]), x[i+128]}; y[i] = tanf_finish_u35(x[i+192], s); }
K1(p32_exp, float, expf_u10(v))
K1(p32_exp2, float, exp2f_u10(v))
K1(p32_log, float, logf_u10(v))
K1(p32_log2, float, log2f_u10(v))
K1(p32_sinh, float, sinhf_u10(v))
K1(p32_cosh, float, coshf_u10(v))
K1(p32_tanh, float, tanhf_u10(v))
K1(p32_log35, float, logf_u35(v))
K1(p32_asin, float, asinf_u10(v))
K1(p32_asin35, float, asinf_u35(v))
K1(p32_acos, float, acosf_u10(v))
K1(p32_acos35, float, acosf_u35(v))
K1(p32_atan, float, atanf_u10(v))
K1(p32_atan35, float, atanf_u35(v))
__global__ void p32_pow(const float* x, float* y) { int i = threadIdx.x; y[i] = powf_u10(x[i], x[i+64]); }
__global__ void p32_atan2(const float* x, float* y) { int i = threadIdx.x; y[i] = atan2f_u10(x[i], x[i+64]); }
__global__ void p32_hypot(const float* x, float* y) { int i = threadIdx.x; y[i] = hypotf_u10(x[i], x[i+64]); }
__global__ void p32_atan235(const float* x, float* y) { int i = threadIdx.x; y[i] = atan2f_u35(x[i], x[i+64]); }
__global__ void p32_pow35(const float* x, float* y) { int i = threadIdx.x; y[i] = powf_u35(x[i], x[i+64]); }
K1(p32_sinh35, float, sinhf_u35(v))
K1(p32_cosh35, float, coshf_u35(v))
K1(p32_tanh35, float, tanhf_u35(v))
K1(p32_log10, float, log10f_u10(v))
K1(p32_log1p, float, log1pf_u10(v))
K1(p32_exp10, float, exp10f_u10(v))
K1(p32_expm1, float, expm1f_u10(v))
K1(p32_cbrt, float, cbrtf_u10(v))
K1(p32_asinh, float, asinhf_u10(v))
K1(p32_acosh, float, acoshf_u10(v))
K1(p32_atanh, float, atanhf_u10(v))
K1(p32_erf, float, erff_u10(v))
K1(p32_erfc, float, erfcf_u10(v))
// exact remainders: the whole functions (one copy of the digit step) and
// one digit step alone
__global__ void p64_fmod(const double* x, double* y) { int i = threadIdx.x; y[i] = fmod_f64(x[i], x[i+64]); }
__global__ void p64_remainder(const double* x, double* y) { int i = threadIdx.x; y[i] = remainder_f64(x[i], x[i+64]); }
__global__ void p64_fmodstep(const double* x, double* y) { int i = threadIdx.x; ddd r = fmod_step(mk(x[i], x[i+64]), x[i+128], x[i+192], x[i+256], (int)x[i+320]); y[i] = r.hi + r.lo; }
__global__ void p32_fmod(const float* x, float* y) { int i = threadIdx.x; y[i] = fmodf_f32(x[i], x[i+64]); }
__global__ void p32_remainder(const float* x, float* y) { int i = threadIdx.x; y[i] = remainderf_f32(x[i], x[i+64]); }
__global__ void p32_fmodstep(const float* x, float* y) { int i = threadIdx.x; fff r = fmodf_step(mk(x[i], x[i+64]), x[i+128], x[i+192], x[i+256], (int)x[i+320]); y[i] = r.hi + r.lo; }
