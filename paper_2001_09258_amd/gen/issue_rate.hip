// VALU issue-rate measurement on gfx950: every lane runs 8 independent
// chains of one instruction kind (or FP64 FMAs interleaved with another
// kind) for 512 steps over 8192 workgroups of 256 lanes, timed with HIP
// events; prints lane-instructions per second against the 39.3 T/s of
// 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.  It supports the VALU roofline the
// benchmark reports; the library does not use it.
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops //         -o issue_rate issue_rate.hip && ./issue_rate
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#define CHK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s line %d\n", hipGetErrorString(e), __LINE__); exit(1); } } while (0)
constexpr int CH = 8, IT = 512;
template <class T, class F>
__global__ __launch_bounds__(256) void k(T* out, T a, T b, F f) {
  T v[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) v[c] = (T)(threadIdx.x + c) * a;
  for (int i = 0; i < IT; ++i) {
#pragma unroll
    for (int c = 0; c < CH; ++c) v[c] = f(v[c], a, b);
  }
  T s = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += v[c];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
struct FmaD { __device__ double operator()(double x, double a, double b) const { return __builtin_fma(x, a, b); } };
struct AddD { __device__ double operator()(double x, double a, double b) const { return x + a; } };
struct MulD { __device__ double operator()(double x, double a, double b) const { return x * a; } };
struct RintD { __device__ double operator()(double x, double a, double b) const { return __builtin_rint(x) + 0.0 * a; } };
struct LdexpD { __device__ double operator()(double x, double a, double b) const { return __builtin_amdgcn_ldexp(x, (int)b); } };
struct FmaF { __device__ float operator()(float x, float a, float b) const { return __builtin_fmaf(x, a, b); } };
struct AddF { __device__ float operator()(float x, float a, float b) const { return x + a; } };
// two independent instructions per step: FP64 FMA and 32-bit integer add on the bits
struct CmpSelD { __device__ double operator()(double x, double a, double b) const { return x > a ? x - b : x + b; } };
// FP64 FMA chains interleaved with independent chains of another kind
template <int KIND>
__global__ __launch_bounds__(256) void kmix(double* out, double a, double b, unsigned ia, float fa) {
  double v[CH];
  unsigned w[CH];
  float f[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) { v[c] = (double)(threadIdx.x + c) * a; w[c] = threadIdx.x * 7u + c; f[c] = (float)(threadIdx.x + c); }
  for (int i = 0; i < IT; ++i) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      v[c] = __builtin_fma(v[c], a, b);
      if (KIND == 0) w[c] = (w[c] ^ ia) + 0x9e3779b9u;      // two 32-bit integer ops
      if (KIND == 1) f[c] = __builtin_fmaf(f[c], fa, 1e-3f);  // one FP32 FMA
    }
  }
  double s = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += v[c] + (double)w[c] + (double)f[c];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
template <int KIND>
void runmix(const char* name, int extra) {
  int blocks = 256 * 32;
  double* out;
  CHK(hipMalloc(&out, sizeof(double) * blocks * 256));
  hipEvent_t e0, e1;
  CHK(hipEventCreate(&e0)); CHK(hipEventCreate(&e1));
  hipLaunchKernelGGL((kmix<KIND>), dim3(blocks), dim3(256), 0, 0, out, 1.0000001, 1e-7, 5u, 1.0001f);
  CHK(hipGetLastError());
  CHK(hipEventRecord(e0, 0));
  for (int r = 0; r < 5; ++r) hipLaunchKernelGGL((kmix<KIND>), dim3(blocks), dim3(256), 0, 0, out, 1.0000001, 1e-7, 5u, 1.0001f);
  CHK(hipEventRecord(e1, 0));
  CHK(hipEventSynchronize(e1));
  float ms; CHK(hipEventElapsedTime(&ms, e0, e1)); ms /= 5;
  double lane = (double)blocks * 256 * CH * IT;
  printf("%-10s %8.3f ms  f64 fma %6.2f T/s + other %6.2f T/s, total %.2f x 39.3\n", name, ms,
         lane / (ms * 1e-3) / 1e12, extra * lane / (ms * 1e-3) / 1e12, (1 + extra) * lane / (ms * 1e-3) / 39.32e12);
  CHK(hipFree(out));
}
template <class T, class F>
void run(const char* name, int ninstr_per_step) {
  int blocks = 256 * 32;
  T* out;
  CHK(hipMalloc(&out, sizeof(T) * blocks * 256));
  hipEvent_t e0, e1;
  CHK(hipEventCreate(&e0)); CHK(hipEventCreate(&e1));
  hipLaunchKernelGGL((k<T, F>), dim3(blocks), dim3(256), 0, 0, out, (T)1.0000001, (T)1e-7, F());
  CHK(hipGetLastError());
  CHK(hipEventRecord(e0, 0));
  for (int r = 0; r < 5; ++r) hipLaunchKernelGGL((k<T, F>), dim3(blocks), dim3(256), 0, 0, out, (T)1.0000001, (T)1e-7, F());
  CHK(hipEventRecord(e1, 0));
  CHK(hipEventSynchronize(e1));
  float ms; CHK(hipEventElapsedTime(&ms, e0, e1)); ms /= 5;
  double lane_ops = (double)blocks * 256 * CH * IT * ninstr_per_step;
  printf("%-10s %8.3f ms  %6.2f T lane-instr/s (%.2f x 39.3)\n", name, ms, lane_ops / (ms * 1e-3) / 1e12,
         lane_ops / (ms * 1e-3) / 39.32e12);
  CHK(hipFree(out));
}
int main() {
  run<double, FmaD>("fma_f64", 1);
  run<double, AddD>("add_f64", 1);
  run<double, MulD>("mul_f64", 1);
  run<double, RintD>("rint+add", 2);
  run<double, LdexpD>("ldexp_f64", 1);
  run<double, CmpSelD>("cmp+2sel+add", 4);
  runmix<0>("fma64+2int", 2);
  runmix<1>("fma64+fma32", 1);
  run<float, FmaF>("fma_f32", 1);
  run<float, AddF>("add_f32", 1);
  return 0;
}
