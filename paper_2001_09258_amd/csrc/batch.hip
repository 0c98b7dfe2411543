// Batched evaluation: one persistent kernel serves a list of requests
// (function, variant, element type, arrays, n) of uneven lengths.
//
// Not part of the paper.  The requests are cut into tiles of TILE elements;
// workgroups take tiles from a device counter until none is left, so long
// and short requests share the machine without one launch per request.  The
// host orders requests by estimated cost (elements x per-element work, most
// expensive first) before numbering their tiles, so the costly tiles start
// early and the tail of the batch is made of cheap ones.  Dispatch on the
// request's operation is uniform across the workgroup.
//
// A plan owns the device copy of the request table and the tile counter, and
// a hip graph of [counter reset kernel -> persistent kernel] captured on
// first use: every run uploads the table and replays the graph.  The kernel
// reads the table and the tile total from device memory, so the graph stays
// valid for any request list that fits the plan.
#include "ops.h"
#include "abi_util.h"
#include "../../include/libm_hip.h"

#include <algorithm>
#include <mutex>
#include <new>
#include <stdio.h>
#include <string.h>
#include <vector>

namespace {
using namespace lmh_ops;

constexpr int BBLOCK = 256;
constexpr int TILE = 4096;          // elements per tile (16 per lane)
constexpr int MAX_REQ = 1024;       // requests per plan

struct Desc {
  const void* a;
  const void* b;
  void* out;
  unsigned long long n;
  unsigned long long tile_begin;
  int op;
  int pad;
};

struct Header {
  unsigned long long total_tiles;
  int k;
  int pad;
};

// ---- operation table -------------------------------------------------------
// X(code, Io, Op, arity)
#define LMH_BATCH_OPS(X)                                                       \
  X(0, IoF64, OpSinU10, 1) X(1, IoF32, OpSinU10, 1) X(2, IoBF16, OpSinU10, 1)    \
  X(3, IoF16, OpSinU10, 1) X(4, IoF32ViaF64, OpSinU10, 1)                       \
  X(5, IoF64, OpSinU35, 1) X(6, IoF32, OpSinU35, 1)                             \
  X(7, IoF64, OpCosU10, 1) X(8, IoF32, OpCosU10, 1) X(9, IoBF16, OpCosU10, 1)    \
  X(10, IoF16, OpCosU10, 1) X(11, IoF32ViaF64, OpCosU10, 1)                     \
  X(12, IoF64, OpCosU35, 1) X(13, IoF32, OpCosU35, 1)                           \
  X(14, IoF64, OpTanU10, 1) X(15, IoF32, OpTanU10, 1) X(16, IoBF16, OpTanU10, 1) \
  X(17, IoF16, OpTanU10, 1) X(18, IoF32ViaF64, OpTanU10, 1)                     \
  X(19, IoF64, OpTanU35, 1) X(20, IoF32, OpTanU35, 1)                           \
  X(21, IoF64, OpExpU10, 1) X(22, IoF32, OpExpU10, 1) X(23, IoBF16, OpExpU10, 1) \
  X(24, IoF16, OpExpU10, 1) X(25, IoF32ViaF64, OpExpU10, 1)                     \
  X(26, IoF64, OpExp2U10, 1) X(27, IoF32, OpExp2U10, 1) X(28, IoBF16, OpExp2U10, 1) \
  X(29, IoF16, OpExp2U10, 1) X(30, IoF32ViaF64, OpExp2U10, 1)                   \
  X(31, IoF64, OpLogU10, 1) X(32, IoF32, OpLogU10, 1) X(33, IoBF16, OpLogU10, 1) \
  X(34, IoF16, OpLogU10, 1) X(35, IoF32ViaF64, OpLogU10, 1)                     \
  X(36, IoF64, OpLog2U10, 1) X(37, IoF32, OpLog2U10, 1) X(38, IoBF16, OpLog2U10, 1) \
  X(39, IoF16, OpLog2U10, 1) X(40, IoF32ViaF64, OpLog2U10, 1)                   \
  X(41, IoF64, OpSinhU10, 1) X(42, IoF32, OpSinhU10, 1) X(43, IoBF16, OpSinhU10, 1) \
  X(44, IoF16, OpSinhU10, 1) X(45, IoF32ViaF64, OpSinhU10, 1)                   \
  X(46, IoF64, OpCoshU10, 1) X(47, IoF32, OpCoshU10, 1) X(48, IoBF16, OpCoshU10, 1) \
  X(49, IoF16, OpCoshU10, 1) X(50, IoF32ViaF64, OpCoshU10, 1)                   \
  X(51, IoF64, OpTanhU10, 1) X(52, IoF32, OpTanhU10, 1) X(53, IoBF16, OpTanhU10, 1) \
  X(54, IoF16, OpTanhU10, 1) X(55, IoF32ViaF64, OpTanhU10, 1)                   \
  X(56, IoF64, OpPowU10, 2) X(57, IoF32, OpPowU10, 2) X(58, IoBF16, OpPowU10, 2) \
  X(59, IoF16, OpPowU10, 2) X(60, IoF32ViaF64, OpPowU10, 2)                     \
  X(61, IoF64, OpAtan2U10, 2) X(62, IoF32, OpAtan2U10, 2) X(63, IoBF16, OpAtan2U10, 2) \
  X(64, IoF16, OpAtan2U10, 2) X(65, IoF32ViaF64, OpAtan2U10, 2)                 \
  X(66, IoF64, OpFmod, 2) X(67, IoF32, OpFmod, 2)                               \
  X(68, IoF64, OpRemainder, 2) X(69, IoF32, OpRemainder, 2)                     \
  X(70, IoF64, OpAsinU10, 1) X(71, IoF32, OpAsinU10, 1) X(72, IoBF16, OpAsinU10, 1) \
  X(73, IoF16, OpAsinU10, 1) X(74, IoF32ViaF64, OpAsinU10, 1)                   \
  X(75, IoF64, OpAsinU35, 1) X(76, IoF32, OpAsinU35, 1)                         \
  X(77, IoF64, OpAcosU10, 1) X(78, IoF32, OpAcosU10, 1) X(79, IoBF16, OpAcosU10, 1) \
  X(80, IoF16, OpAcosU10, 1) X(81, IoF32ViaF64, OpAcosU10, 1)                   \
  X(82, IoF64, OpAcosU35, 1) X(83, IoF32, OpAcosU35, 1)                         \
  X(84, IoF64, OpAtanU10, 1) X(85, IoF32, OpAtanU10, 1) X(86, IoBF16, OpAtanU10, 1) \
  X(87, IoF16, OpAtanU10, 1) X(88, IoF32ViaF64, OpAtanU10, 1)                   \
  X(89, IoF64, OpAtanU35, 1) X(90, IoF32, OpAtanU35, 1)                         \
  X(91, IoF64, OpLogU35, 1) X(92, IoF32, OpLogU35, 1)                           \
  X(93, IoF64, OpLog10U10, 1) X(94, IoF32, OpLog10U10, 1) X(95, IoBF16, OpLog10U10, 1) \
  X(96, IoF16, OpLog10U10, 1) X(97, IoF32ViaF64, OpLog10U10, 1)                 \
  X(98, IoF64, OpLog1pU10, 1) X(99, IoF32, OpLog1pU10, 1) X(100, IoBF16, OpLog1pU10, 1) \
  X(101, IoF16, OpLog1pU10, 1) X(102, IoF32ViaF64, OpLog1pU10, 1)               \
  X(103, IoF64, OpExp10U10, 1) X(104, IoF32, OpExp10U10, 1) X(105, IoBF16, OpExp10U10, 1) \
  X(106, IoF16, OpExp10U10, 1) X(107, IoF32ViaF64, OpExp10U10, 1)               \
  X(108, IoF64, OpExpm1U10, 1) X(109, IoF32, OpExpm1U10, 1) X(110, IoBF16, OpExpm1U10, 1) \
  X(111, IoF16, OpExpm1U10, 1) X(112, IoF32ViaF64, OpExpm1U10, 1)               \
  X(113, IoF64, OpCbrtU10, 1) X(114, IoF32, OpCbrtU10, 1) X(115, IoBF16, OpCbrtU10, 1) \
  X(116, IoF16, OpCbrtU10, 1) X(117, IoF32ViaF64, OpCbrtU10, 1)                 \
  X(118, IoF64, OpHypotU10, 2) X(119, IoF32, OpHypotU10, 2) X(120, IoBF16, OpHypotU10, 2) \
  X(121, IoF16, OpHypotU10, 2) X(122, IoF32ViaF64, OpHypotU10, 2)             \
  X(123, IoF64, OpAtan2U35, 2) X(124, IoF32, OpAtan2U35, 2)                     \
  X(125, IoF64, OpSinhU35, 1) X(126, IoF32, OpSinhU35, 1)                       \
  X(127, IoF64, OpCoshU35, 1) X(128, IoF32, OpCoshU35, 1)                       \
  X(129, IoF64, OpTanhU35, 1) X(130, IoF32, OpTanhU35, 1)                       \
  X(131, IoF64, OpAsinhU10, 1) X(132, IoF32, OpAsinhU10, 1) X(133, IoBF16, OpAsinhU10, 1) \
  X(134, IoF16, OpAsinhU10, 1) X(135, IoF32ViaF64, OpAsinhU10, 1)               \
  X(136, IoF64, OpAcoshU10, 1) X(137, IoF32, OpAcoshU10, 1) X(138, IoBF16, OpAcoshU10, 1) \
  X(139, IoF16, OpAcoshU10, 1) X(140, IoF32ViaF64, OpAcoshU10, 1)               \
  X(141, IoF64, OpAtanhU10, 1) X(142, IoF32, OpAtanhU10, 1) X(143, IoBF16, OpAtanhU10, 1) \
  X(144, IoF16, OpAtanhU10, 1) X(145, IoF32ViaF64, OpAtanhU10, 1)               \
  X(146, IoF64, OpErfU10, 1) X(147, IoF32, OpErfU10, 1) X(148, IoBF16, OpErfU10, 1) \
  X(149, IoF16, OpErfU10, 1) X(150, IoF32ViaF64, OpErfU10, 1)                   \
  X(151, IoF64, OpErfcU10, 1) X(152, IoF32, OpErfcU10, 1) X(153, IoBF16, OpErfcU10, 1) \
  X(154, IoF16, OpErfcU10, 1) X(155, IoF32ViaF64, OpErfcU10, 1)               \
  X(156, IoF64, OpFdim, 2) X(157, IoF32, OpFdim, 2)                             \
  X(158, IoF64, OpFmax, 2) X(159, IoF32, OpFmax, 2)                             \
  X(160, IoF64, OpFmin, 2) X(161, IoF32, OpFmin, 2)                             \
  X(162, IoF64, OpSqrt, 1) X(163, IoF32, OpSqrt, 1) \
  X(164, IoF64, OpTrunc, 1) X(165, IoF32, OpTrunc, 1) \
  X(166, IoF64, OpFloor, 1) X(167, IoF32, OpFloor, 1) \
  X(168, IoF64, OpCeil, 1) X(169, IoF32, OpCeil, 1) \
  X(170, IoF64, OpRound, 1) X(171, IoF32, OpRound, 1) \
  X(172, IoF64, OpRint, 1) X(173, IoF32, OpRint, 1) \
  X(174, IoF64, OpFabs, 1) X(175, IoF32, OpFabs, 1) \
  X(176, IoF64, OpLogb, 1) X(177, IoF32, OpLogb, 1) \
  X(178, IoF64, OpCopysign, 2) X(179, IoF32, OpCopysign, 2) \
  X(180, IoF64, OpNextafter, 2) X(181, IoF32, OpNextafter, 2) \
  X(182, IoF64, OpPowU35, 2) X(183, IoF32, OpPowU35, 2) \
  X(184, IoF64, OpLgammaU10, 1) X(185, IoF32, OpLgammaU10, 1) X(186, IoBF16, OpLgammaU10, 1) \
  X(187, IoF16, OpLgammaU10, 1) X(188, IoF32ViaF64, OpLgammaU10, 1)               \
  X(189, IoF64, OpTgammaU10, 1) X(190, IoF32, OpTgammaU10, 1) X(191, IoBF16, OpTgammaU10, 1) \
  X(192, IoF16, OpTgammaU10, 1) X(193, IoF32ViaF64, OpTgammaU10, 1)
constexpr int NUM_OPS = 194;

// host-side code of a (fn, variant, dtype) triple, or -1
int op_code(int fn, int v, int t) {
  // dtype order in the table: f64, f32, bf16, f16, f32_via_f64
  static const int u10_base[LIBM_HIP_NUM_FN] = {0, 7, 14, 21, 26, 31, 36, 56, 61, 41, 46, 51,
                                                -1, -1, 70, 77, 84, 93, 98, 103, 108, 113,
                                                118, 131, 136, 141, 146, 151, -1, -1, -1,
                                                -1, -1, -1, -1, -1, -1, -1, -1, -1, -1,
                                                184, 189};
  static const int u35_base[LIBM_HIP_NUM_FN] = {5, 12, 19, -1, -1, 91, -1, 182, 123, 125, 127,
                                                129, -1, -1, 75, 82, 89, -1, -1, -1, -1, -1,
                                                -1, -1, -1, -1, -1, -1, -1, -1, -1,
                                                -1, -1, -1, -1, -1, -1, -1, -1, -1, -1,
                                                -1, -1};
  if (fn < 0 || fn >= LIBM_HIP_NUM_FN || t < 0 || t > 4) return -1;
  if (fn == LIBM_HIP_FMOD || fn == LIBM_HIP_REMAINDER) {
    if (v != LIBM_HIP_EXACT || t > 1) return -1;
    return (fn == LIBM_HIP_FMOD ? 66 : 68) + t;
  }
  if (fn >= LIBM_HIP_FDIM && fn <= LIBM_HIP_NEXTAFTER) {          // exact, f64 and f32
    if (v != LIBM_HIP_EXACT || t > 1) return -1;
    return 156 + 2 * (fn - LIBM_HIP_FDIM) + t;
  }
  if (v == LIBM_HIP_U10) return u10_base[fn] + t;
  if (v == LIBM_HIP_U35) return u35_base[fn] < 0 || t > 1 ? -1 : u35_base[fn] + t;
  return -1;
}

// relative per-element cost used to order requests, by function family
// (from the elementwise kernels' measured times: trig with Payne-Hanek and
// the remainders are the most expensive, exp/log the cheapest)
float op_cost(int code) {
  if (code >= 184) return 1.5f;                // lgamma, tgamma
  if (code >= 182) return 0.75f;               // pow u35
  if (code >= 156) return 0.25f;               // fdim, fmax, fmin and the rest of the exact set
  if (code >= 146) return 0.5f;                // erf, erfc
  if (code >= 131) return 0.55f;               // asinh, acosh, atanh
  if (code >= 125) return 0.35f;               // sinh, cosh, tanh u35
  if (code >= 123) return 0.5f;                // atan2 u35
  if (code >= 113) return 0.45f;               // cbrt, hypot
  if (code >= 93) return 0.4f;                 // log10, log1p, exp10, expm1
  if (code >= 91) return 0.3f;                 // log u35
  if (code >= 70) return 0.6f;                 // asin, acos, atan
  if (code >= 66) return 1.5f;                 // fmod, remainder
  if (code <= 20) return 1.0f;                 // sin, cos, tan
  if (code >= 56) return 0.8f;                 // pow, atan2
  if (code >= 41) return 0.5f;                 // sinh, cosh, tanh
  return 0.35f;                                // exp, exp2, log, log2
}

size_t op_arity(int code) {
  return (code >= 56 && code <= 69) || (code >= 118 && code <= 124) ||
                 (code >= 156 && code <= 161) || (code >= 178 && code <= 183)
             ? 2
             : 1;
}

// ---- device side -------------------------------------------------------------
// One tile of one request.  Kept out of line: each operation's tile loop is
// register-allocated on its own, so the persistent kernel is not charged the
// union of all seventy bodies (inlined, the switch needed 199 VGPRs and ran
// at two waves per SIMD).  A full tile of 16-byte aligned arrays moves
// 16-byte packs like the elementwise kernels; anything else goes element by
// element.
template <class Io, class Op, int ARITY>
__device__ __noinline__ void run_tile(const void* av, const void* bv, void* yv,
                                      unsigned long long n, unsigned long long start) {
  typedef typename Io::S S;
  constexpr int EPT = ept_for<S>();
  const S* a = (const S*)av;
  const S* b = (const S*)bv;
  S* y = (S*)yv;
  unsigned long long end = start + TILE < n ? start + TILE : n;
  uintptr_t al = (uintptr_t)a | (uintptr_t)y | (ARITY == 2 ? (uintptr_t)b : 0);
  if ((al & 15u) == 0 && end - start == TILE) {
    for (int p = threadIdx.x; p < TILE / EPT; p += BBLOCK) {
      unsigned long long base = start + (unsigned long long)p * EPT;
      Pack<S, EPT> ia = *reinterpret_cast<const Pack<S, EPT>*>(a + base);
      Pack<S, EPT> o;
      if constexpr (ARITY == 1) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) o.v[i] = Io::out(Op::f(Io::in(ia.v[i])));
      } else {
        Pack<S, EPT> ib = *reinterpret_cast<const Pack<S, EPT>*>(b + base);
#pragma unroll
        for (int i = 0; i < EPT; ++i) o.v[i] = Io::out(Op::f(Io::in(ia.v[i]), Io::in(ib.v[i])));
      }
      store_nt(o, y + base);
    }
    return;
  }
  for (unsigned long long i = start + threadIdx.x; i < end; i += BBLOCK) {
    if constexpr (ARITY == 1)
      y[i] = Io::out(Op::f(Io::in(a[i])));
    else
      y[i] = Io::out(Op::f(Io::in(a[i]), Io::in(b[i])));
  }
}

__global__ void k_batch_reset(unsigned long long* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0ull;
}

__global__ __launch_bounds__(BBLOCK) __attribute__((amdgpu_waves_per_eu(6)))
void k_batch(const Desc* __restrict__ descs,
                                                  const Header* __restrict__ hdr,
                                                  unsigned long long* counter) {
  __shared__ unsigned long long s_tile;
  const unsigned long long total = hdr->total_tiles;
  const int k = hdr->k;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1ull);
    __syncthreads();
    unsigned long long t = s_tile;
    __syncthreads();
    if (t >= total) break;                   // the counter only grows: every
                                             // workgroup reaches this exit
    // request owning tile t: last r with tile_begin <= t (binary search)
    int lo = 0, hi = k - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (descs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    Desc d = descs[lo];
    unsigned long long start = (t - d.tile_begin) * (unsigned long long)TILE;
    switch (d.op) {
#define LMH_CASE(code, Io, Op, ar) \
  case code: run_tile<Io, typename EvalOp<Io, Op>::type, ar>(d.a, d.b, d.out, d.n, start); break;
      LMH_BATCH_OPS(LMH_CASE)
#undef LMH_CASE
      default: break;
    }
  }
}

// ---- the no-allocation form ---------------------------------------------------
// libm_hip_batch_run_noalloc keeps its request table, header and tile counter
// in this file-scope device array instead of plan memory: every GPU the
// library runs on holds one copy until the process ends.  Layout: tile
// counter at byte 0, header at byte 64, request table from byte 256.  Host
// code never uses the array's name as an address (in host code it names a
// host-side stand-in); it uses the device address hipGetSymbolAddress gives
// for the current device, kept per device.
constexpr int NOALLOC_MAX_REQ = 256;
constexpr size_t SCRATCH_TABLE = 256;
constexpr size_t SCRATCH_BYTES = SCRATCH_TABLE + sizeof(Desc) * NOALLOC_MAX_REQ;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// the staging kernel takes up to STAGE_CHUNK descriptors by value (kernel
// arguments, no host-to-device copy) and writes them into the table; the
// launch that stages the first chunk also writes the header and clears the
// tile counter
constexpr int STAGE_CHUNK = 64;
struct StageArgs {
  Desc d[STAGE_CHUNK];
  Header h;
  int first;
  int count;
};
static_assert(sizeof(StageArgs) < 4000, "kernel arguments stay below 4 KiB");

__global__ void k_batch_stage(StageArgs args, unsigned char* base) {
  Desc* table = reinterpret_cast<Desc*>(base + SCRATCH_TABLE);
  int i = threadIdx.x;
  if (i < args.count) table[args.first + i] = args.d[i];
  if (args.first == 0 && i == 0) {
    *reinterpret_cast<Header*>(base + 64) = args.h;
    *reinterpret_cast<unsigned long long*>(base) = 0ull;
  }
}

// batch errors go to the library's one thread-local message
void batch_error(const char* m) { lmh_abi::set_error(m); }

// makes `device` current for the lifetime of the guard (device < 0: keep the
// current one) and restores the previous current device afterwards
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int device) {
    if (device < 0) return;
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != device) err = hipSetDevice(device);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct libm_hip_batch_plan {
  int device;
  int max_requests;
  Desc* d_descs;
  Header* d_hdr;
  unsigned long long* d_counter;
  Desc* h_descs;          // pinned staging
  Header* h_hdr;
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipStream_t capture_stream;   // private stream used only to capture the graph
  hipEvent_t staged;            // the last upload from the pinned table is done
  bool staged_valid;
  unsigned grid;
  bool use_graph;
};

extern "C" {

const char* libm_hip_batch_last_error(void) { return lmh_abi::g_last_error; }

libm_hip_status libm_hip_batch_plan_create(libm_hip_batch_plan** out, int max_requests,
                                           int device) {
  int ndev = 0;
  if (!out || max_requests <= 0 || max_requests > MAX_REQ ||
      (device >= 0 && (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev))) {
    batch_error("libm_hip_batch_plan_create: invalid arguments (1 <= max_requests <= 1024, "
                "device -1 or an existing device)");
    return LIBM_HIP_ERR_INVALID;
  }
  DeviceGuard guard(device);
  if (guard.err != hipSuccess) {
    batch_error(hipGetErrorString(guard.err));
    return LIBM_HIP_ERR_HIP;
  }
  libm_hip_batch_plan* p = new (std::nothrow) libm_hip_batch_plan();
  if (!p) {
    batch_error("libm_hip_batch_plan_create: out of host memory");
    return LIBM_HIP_ERR_NOMEM;
  }
  memset(p, 0, sizeof(*p));
  p->max_requests = max_requests;
  p->use_graph = true;
  hipError_t e = hipGetDevice(&p->device);
  int cus = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_descs, sizeof(Desc) * max_requests);
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_hdr, sizeof(Header));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_counter, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_descs, sizeof(Desc) * max_requests, 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_hdr, sizeof(Header), 0);
  if (e == hipSuccess) e = hipStreamCreate(&p->capture_stream);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->staged, hipEventDisableTiming);
  if (e != hipSuccess) {
    batch_error(hipGetErrorString(e));
    libm_hip_batch_plan_destroy(p);
    return LIBM_HIP_ERR_NOMEM;
  }
  // one resident wave of workgroups: as many per CU as the kernel's
  // registers allow (a persistent workgroup beyond that would only start
  // once the queue is empty)
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, BBLOCK, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 4;
  p->grid = (unsigned)((cus > 0 ? cus : 256) * per_cu);
  *out = p;
  return LIBM_HIP_OK;
}

libm_hip_status libm_hip_batch_plan_set_graph(libm_hip_batch_plan* p, int use_graph) {
  if (!p) {
    batch_error("libm_hip_batch_plan_set_graph: NULL plan");
    return LIBM_HIP_ERR_INVALID;
  }
  p->use_graph = use_graph != 0;
  return LIBM_HIP_OK;
}

void libm_hip_batch_plan_destroy(libm_hip_batch_plan* p) {
  if (!p) return;
  DeviceGuard guard(p->device);
  // teardown errors cannot be reported through a void call; they are ignored
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_descs) (void)hipFree(p->d_descs);
  if (p->d_hdr) (void)hipFree(p->d_hdr);
  if (p->d_counter) (void)hipFree(p->d_counter);
  if (p->h_descs) (void)hipHostFree(p->h_descs);
  if (p->h_hdr) (void)hipHostFree(p->h_hdr);
  if (p->staged) (void)hipEventDestroy(p->staged);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  delete p;
}

static hipError_t enqueue_kernels(libm_hip_batch_plan* p, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, p->d_counter);
  hipLaunchKernelGGL(k_batch, dim3(p->grid), dim3(BBLOCK), 0, s, p->d_descs, p->d_hdr,
                     p->d_counter);
  return hipGetLastError();
}

libm_hip_status libm_hip_batch_run(libm_hip_batch_plan* p, const libm_hip_request* reqs, int k,
                                   void* stream) {
  if (!p || (k > 0 && !reqs) || k < 0 || k > p->max_requests) {
    batch_error("libm_hip_batch_run: invalid arguments");
    return LIBM_HIP_ERR_INVALID;
  }
  DeviceGuard guard(p->device);
  if (guard.err != hipSuccess) {
    batch_error(hipGetErrorString(guard.err));
    return LIBM_HIP_ERR_HIP;
  }
  hipStream_t s = (hipStream_t)stream;
  // validate and order by estimated cost, most expensive first
  std::vector<int> order;
  std::vector<float> cost(k);
  std::vector<int> codes(k);
  for (int i = 0; i < k; ++i) {
    const libm_hip_request& r = reqs[i];
    int code = op_code(r.fn, r.variant, r.dtype);
    if (code < 0) {
      batch_error("libm_hip_batch_run: unsupported (fn, variant, dtype)");
      return LIBM_HIP_ERR_UNSUPPORTED;
    }
    if (r.n > 0 && (!r.a || !r.out || (op_arity(code) == 2 && !r.b))) {
      batch_error("libm_hip_batch_run: NULL pointer with n > 0");
      return LIBM_HIP_ERR_INVALID;
    }
    codes[i] = code;
    cost[i] = op_cost(code) * (float)r.n;
    if (r.n > 0) order.push_back(i);
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  if (order.empty()) return LIBM_HIP_OK;
  // the pinned table may still feed the previous run's upload
  hipError_t e = p->staged_valid ? hipEventSynchronize(p->staged) : hipSuccess;
  if (e != hipSuccess) {
    batch_error(hipGetErrorString(e));
    return LIBM_HIP_ERR_HIP;
  }
  unsigned long long tiles = 0;
  int m = 0;
  for (int i : order) {
    const libm_hip_request& r = reqs[i];
    Desc& d = p->h_descs[m++];
    d.a = r.a;
    d.b = r.b;
    d.out = r.out;
    d.n = r.n;
    d.tile_begin = tiles;
    d.op = codes[i];
    d.pad = 0;
    tiles += (r.n + TILE - 1) / TILE;
  }
  p->h_hdr->total_tiles = tiles;
  p->h_hdr->k = m;
  p->h_hdr->pad = 0;
  e = hipMemcpyAsync(p->d_descs, p->h_descs, sizeof(Desc) * m, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->d_hdr, p->h_hdr, sizeof(Header), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(p->staged, s);
  if (e != hipSuccess) {
    batch_error(hipGetErrorString(e));
    return LIBM_HIP_ERR_HIP;
  }
  p->staged_valid = true;
  if (p->use_graph) {
    if (!p->exec) {
      // captured once on the plan's own stream (the caller's may be the null
      // stream, which cannot be captured); replayed on the caller's stream
      e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t e2 = enqueue_kernels(p, p->capture_stream);
        e = hipStreamEndCapture(p->capture_stream, &p->graph);
        if (e == hipSuccess) e = e2;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        batch_error(hipGetErrorString(e));
        return LIBM_HIP_ERR_HIP;
      }
    }
    e = hipGraphLaunch(p->exec, s);
  } else {
    e = enqueue_kernels(p, s);
  }
  if (e != hipSuccess) {
    batch_error(hipGetErrorString(e));
    return LIBM_HIP_ERR_HIP;
  }
  return LIBM_HIP_OK;
}

}  // extern "C"

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[MAX_DEVICES];    // device address of scratch, per device
unsigned g_scratch_grid[MAX_DEVICES];         // persistent grid, per device

// set-up on the first call on a device (with that device current): the
// device address of this device's copy of scratch, and the persistent grid
hipError_t noalloc_setup(int dev, unsigned char** base, unsigned* grid) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    unsigned char* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, BBLOCK, 0) != hipSuccess ||
        per_cu <= 0)
      per_cu = 4;
    g_scratch_grid[dev] = (unsigned)((cus > 0 ? cus : 256) * per_cu);
    g_scratch_ptr[dev] = ptr;
  }
  *base = g_scratch_ptr[dev];
  *grid = g_scratch_grid[dev];
  return hipSuccess;
}
}  // namespace

extern "C" libm_hip_status libm_hip_batch_run_noalloc(const libm_hip_request* reqs, int k,
                                                      void* stream) {
  if ((k > 0 && !reqs) || k < 0) {
    batch_error("libm_hip_batch_run_noalloc: invalid arguments");
    return LIBM_HIP_ERR_INVALID;
  }
  if (k > NOALLOC_MAX_REQ) {
    batch_error("libm_hip_batch_run_noalloc: at most 256 requests per call");
    return LIBM_HIP_ERR_INVALID;
  }
  // validate and order by estimated cost, most expensive first (fixed-size
  // arrays on the stack: no allocation of any kind)
  int order[NOALLOC_MAX_REQ];
  float cost[NOALLOC_MAX_REQ];
  int codes[NOALLOC_MAX_REQ];
  int m = 0;
  for (int i = 0; i < k; ++i) {
    const libm_hip_request& r = reqs[i];
    int code = op_code(r.fn, r.variant, r.dtype);
    if (code < 0) {
      batch_error("libm_hip_batch_run_noalloc: unsupported (fn, variant, dtype)");
      return LIBM_HIP_ERR_UNSUPPORTED;
    }
    if (r.n > 0 && (!r.a || !r.out || (op_arity(code) == 2 && !r.b))) {
      batch_error("libm_hip_batch_run_noalloc: NULL pointer with n > 0");
      return LIBM_HIP_ERR_INVALID;
    }
    codes[i] = code;
    cost[i] = op_cost(code) * (float)r.n;
    if (r.n > 0) order[m++] = i;
  }
  if (m == 0) return LIBM_HIP_OK;
  // ties keep the caller's order, as in libm_hip_batch_run
  std::sort(order, order + m, [&](int x, int y) {
    return cost[x] > cost[y] || (cost[x] == cost[y] && x < y);
  });
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess && (dev < 0 || dev >= MAX_DEVICES)) e = hipErrorInvalidDevice;
  unsigned char* base = nullptr;
  unsigned grid = 0;
  if (e == hipSuccess) e = noalloc_setup(dev, &base, &grid);
  if (e != hipSuccess) {
    batch_error(hipGetErrorString(e));
    return LIBM_HIP_ERR_HIP;
  }
  hipStream_t s = (hipStream_t)stream;
  StageArgs args;
  memset(&args, 0, sizeof(args));
  unsigned long long tiles = 0;
  for (int j = 0; j < m; ++j) {
    const libm_hip_request& r = reqs[order[j]];
    tiles += (r.n + TILE - 1) / TILE;
  }
  args.h.total_tiles = tiles;
  args.h.k = m;
  tiles = 0;
  for (int first = 0; first < m && e == hipSuccess; first += STAGE_CHUNK) {
    int count = m - first < STAGE_CHUNK ? m - first : STAGE_CHUNK;
    for (int j = 0; j < count; ++j) {
      const libm_hip_request& r = reqs[order[first + j]];
      Desc& d = args.d[j];
      d.a = r.a;
      d.b = r.b;
      d.out = r.out;
      d.n = r.n;
      d.tile_begin = tiles;
      d.op = codes[order[first + j]];
      d.pad = 0;
      tiles += (r.n + TILE - 1) / TILE;
    }
    args.first = first;
    args.count = count;
    hipLaunchKernelGGL(k_batch_stage, dim3(1), dim3(STAGE_CHUNK), 0, s, args, base);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(BBLOCK), 0, s,
                       reinterpret_cast<const Desc*>(base + SCRATCH_TABLE),
                       reinterpret_cast<const Header*>(base + 64),
                       reinterpret_cast<unsigned long long*>(base));
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    batch_error(hipGetErrorString(e));
    return LIBM_HIP_ERR_HIP;
  }
  return LIBM_HIP_OK;
}
