// Elementwise kernels (device code; the launchers and the C ABI live in
// kernels.hip).
//
// One lane evaluates EPT consecutive elements per 16-byte pack; arrays whose
// pointers are all 16-byte aligned move data with 128-bit global loads and
// non-temporal 128-bit stores (the elements are touched once); any other
// alignment, and the ragged tail, use scalar accesses.  The per-element work
// is one evaluator from eval_f64.h / eval_f32.h: the paper's vector-of-lanes
// execution becomes one element per GPU lane, and its conditional moves
// become exec-masked selects.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

#include "ops.h"

namespace lmh_kernels {
using namespace lmh_ops;

constexpr int BLOCK = 256;          // workgroup of the gathered-trig kernels
constexpr int MAX_BLOCK = 1024;

// Operations with a rare accurate path (a static member kRare) are evaluated
// in two steps over a pack: the common path for every element, then, if any
// lane of the wave flagged an element, the rare path for the flagged ones.
// The pack's evaluations stay one stretch of code the compiler interleaves.
template <class Op, class = void>
struct HasRare {
  static constexpr bool value = false;
};
template <class Op>
struct HasRare<Op, std::void_t<decltype(Op::kRare)>> {
  static constexpr bool value = Op::kRare;
};

template <class Io, class Op, int EPT, class S>
__device__ __forceinline__ void eval_pack1(const Pack<S, EPT>& in, Pack<S, EPT>& out) {
  if constexpr (HasRare<Op>::value) {
    bool rare[EPT];
    bool any = false;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      out.v[i] = Io::out(Op::main(Io::in(in.v[i]), rare[i]));
      any = any || rare[i];
    }
    if (lmh::rare_lane(any)) {
#pragma unroll
      for (int i = 0; i < EPT; ++i)
        if (rare[i]) out.v[i] = Io::out(Op::rare(Io::in(in.v[i])));
    }
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i) out.v[i] = Io::out(Op::f(Io::in(in.v[i])));
  }
}

template <class Io, class Op, int EPT, class S>
__device__ __forceinline__ void eval_pack2(const Pack<S, EPT>& ia, const Pack<S, EPT>& ib,
                                           Pack<S, EPT>& out) {
  if constexpr (HasRare<Op>::value) {
    bool rare[EPT];
    bool any = false;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      out.v[i] = Io::out(Op::main(Io::in(ia.v[i]), Io::in(ib.v[i]), rare[i]));
      any = any || rare[i];
    }
    if (lmh::rare_lane(any)) {
#pragma unroll
      for (int i = 0; i < EPT; ++i)
        if (rare[i]) out.v[i] = Io::out(Op::rare(Io::in(ia.v[i]), Io::in(ib.v[i])));
    }
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i) out.v[i] = Io::out(Op::f(Io::in(ia.v[i]), Io::in(ib.v[i])));
  }
}

// Each workgroup covers blockDim.x * PACKS packs; pack u of a lane is
// (block_base + u * blockDim.x + lane), so every iteration is one fully
// coalesced workgroup-wide access.  Misaligned arrays use PACKS = 1.
template <class Io, class Op, int EPT, bool VEC, int PACKS>
__global__ __launch_bounds__(MAX_BLOCK) void k_unary(const typename Io::S* __restrict__ x,
                                                     typename Io::S* __restrict__ y, size_t n) {
  typedef typename Io::S S;
  size_t pk0 = (size_t)blockIdx.x * blockDim.x * PACKS + threadIdx.x;
#pragma unroll
  for (int u = 0; u < PACKS; ++u) {
    size_t base = (pk0 + (size_t)u * blockDim.x) * EPT;
    if (base >= n) return;
    if (VEC && base + EPT <= n) {
      Pack<S, EPT> in = *reinterpret_cast<const Pack<S, EPT>*>(x + base);
      Pack<S, EPT> out;
      eval_pack1<Io, Op, EPT>(in, out);
      store_nt(out, y + base);
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        if (base + i < n) y[base + i] = Io::out(Op::f(Io::in(x[base + i])));
      }
    }
  }
}

template <class Io, class Op, int EPT, bool VEC, int PACKS>
__global__ __launch_bounds__(MAX_BLOCK) void k_binary(const typename Io::S* __restrict__ a,
                                                      const typename Io::S* __restrict__ b,
                                                      typename Io::S* __restrict__ y, size_t n) {
  typedef typename Io::S S;
  size_t pk0 = (size_t)blockIdx.x * blockDim.x * PACKS + threadIdx.x;
#pragma unroll
  for (int u = 0; u < PACKS; ++u) {
    size_t base = (pk0 + (size_t)u * blockDim.x) * EPT;
    if (base >= n) return;
    if (VEC && base + EPT <= n) {
      Pack<S, EPT> ia = *reinterpret_cast<const Pack<S, EPT>*>(a + base);
      Pack<S, EPT> ib = *reinterpret_cast<const Pack<S, EPT>*>(b + base);
      Pack<S, EPT> out;
      eval_pack2<Io, Op, EPT>(ia, ib, out);
      store_nt(out, y + base);
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        if (base + i < n) y[base + i] = Io::out(Op::f(Io::in(a[base + i]), Io::in(b[base + i])));
      }
    }
  }
}

// Trigonometric kernels with the Payne-Hanek lanes gathered.  Every lane runs
// the Cody-Waite reduction on its elements; the Payne-Hanek ones are also
// written to a workgroup queue in LDS and reduced densely by all lanes after
// a barrier, so a wave that holds a few large arguments no longer pays the
// whole Payne-Hanek path.  Each wave owns a fixed region of the queue and
// fills its front with ballot + mbcnt (no atomics); the dense pass maps its
// index onto the filled fronts from the per-wave counts.  The reduced states
// come back through LDS and every lane finishes its own elements.
constexpr int SPLIT_WAVES = BLOCK / 64;

// Append this lane's slow elements to its wave's region (all lanes of the
// workgroup must call it); the wave's count goes to q_cnt[wave].
template <int EPT, class C>
__device__ __forceinline__ void queue_slow(const C (&xv)[EPT], const bool (&slow)[EPT], C* q_x,
                                           unsigned short* q_slot, unsigned* q_cnt) {
  const unsigned lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  unsigned filled = 0;                               // wave-uniform
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    unsigned long long m = __builtin_amdgcn_ballot_w64(slow[i]);
    unsigned pre = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                             __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
    if (slow[i]) {
      unsigned pos = wave * (64u * EPT) + filled + pre;
      q_x[pos] = xv[i];
      q_slot[pos] = (unsigned short)(threadIdx.x * EPT + i);
    }
    filled += (unsigned)__popcll(m);
  }
  if (lane == 0) q_cnt[wave] = filled;
}

// After a barrier: every queued element reduced once, by the workgroup's
// lanes in dense order, its state stored at its slot.
template <int EPT, class C, class R, class F>
__device__ __forceinline__ void reduce_queue(const C* q_x, const unsigned short* q_slot,
                                             const unsigned* q_cnt, R* q_res, F reduce) {
  unsigned cnt[SPLIT_WAVES], first[SPLIT_WAVES];
  unsigned total = 0;
#pragma unroll
  for (int w = 0; w < SPLIT_WAVES; ++w) {
    cnt[w] = q_cnt[w];
    first[w] = total;
    total += cnt[w];
  }
  for (unsigned p = threadIdx.x; p < total; p += BLOCK) {
    // dense index p -> slot in its wave's region, skipping the unfilled
    // tails of the regions before it
    unsigned pos = p;
#pragma unroll
    for (int w = 1; w < SPLIT_WAVES; ++w) pos += p >= first[w] ? 64u * EPT - cnt[w - 1] : 0u;
    q_res[q_slot[pos]] = reduce(q_x[pos]);
  }
}

// EPT elements of this lane: a 16-byte pack or masked scalar loads
template <class Io, int EPT, bool VEC>
__device__ __forceinline__ void load_lane(const typename Io::S* __restrict__ x, size_t n,
                                          size_t base, typename Io::C (&xv)[EPT],
                                          bool (&ok)[EPT]) {
  typedef typename Io::S S;
  typedef typename Io::C C;
  if (VEC && base + EPT <= n) {
    Pack<S, EPT> in = *reinterpret_cast<const Pack<S, EPT>*>(x + base);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      xv[i] = Io::in(in.v[i]);
      ok[i] = true;
    }
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      ok[i] = base + i < n;
      xv[i] = ok[i] ? Io::in(x[base + i]) : C(0);
    }
  }
}

template <class Io, class Op, int EPT, bool VEC>
__global__ __launch_bounds__(BLOCK) void k_unary_split(const typename Io::S* __restrict__ x,
                                                       typename Io::S* __restrict__ y, size_t n) {
  typedef typename Io::S S;
  typedef typename Io::C C;
  typedef decltype(Op::fast(C())) St;
  __shared__ C q_x[BLOCK * EPT];
  __shared__ unsigned short q_slot[BLOCK * EPT];
  __shared__ St q_res[BLOCK * EPT];
  __shared__ unsigned q_cnt[SPLIT_WAVES];
  size_t base = ((size_t)blockIdx.x * BLOCK + threadIdx.x) * EPT;
  C xv[EPT];
  bool ok[EPT];
  load_lane<Io, EPT, VEC>(x, n, base, xv, ok);
  St st[EPT];
  bool slow[EPT];
  // Cody-Waite for every element, without a branch: nearly every wave holds
  // Cody-Waite elements anyway, and straight-line code lets the compiler
  // interleave the EPT independent reductions (the slow elements' states
  // are replaced below)
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    slow[i] = ok[i] && Op::is_slow(xv[i]);
    st[i] = Op::fast(xv[i]);
  }
  queue_slow<EPT>(xv, slow, q_x, q_slot, q_cnt);
  __syncthreads();
  reduce_queue<EPT>(q_x, q_slot, q_cnt, q_res, [](C v) { return Op::slow(v); });
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i)
    if (slow[i]) st[i] = q_res[threadIdx.x * EPT + i];
  if (VEC && base + EPT <= n) {
    Pack<S, EPT> out;
#pragma unroll
    for (int i = 0; i < EPT; ++i) out.v[i] = Io::out(Op::finish(xv[i], st[i]));
    store_nt(out, y + base);
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (ok[i]) y[base + i] = Io::out(Op::finish(xv[i], st[i]));
  }
}

// The same gathering for the binary64 evaluators, done per wave instead of
// per workgroup: a wave takes WPACKS 16-byte packs per lane, compacts its
// Cody-Waite elements at the front of its own LDS region and its
// Payne-Hanek elements at the back, and then evaluates the region densely,
// 64 elements per step, reduction and finish together; only the one step
// where the two kinds meet runs both reductions.  Each result overwrites its
// input's position (that position is read and written by one lane in one
// step), and the lanes read their results back from the positions they
// wrote.  A wave only reads LDS that its own lanes wrote, so no workgroup
// barrier is needed: wave_lds_sync keeps the compiler from moving LDS
// accesses across it, and one wave's LDS accesses complete in order.
constexpr int WPACKS = 4;

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class Io, class Op, int EPT, bool VEC>
__global__ __launch_bounds__(BLOCK) void k_unary_wsplit(const typename Io::S* __restrict__ x,
                                                        typename Io::S* __restrict__ y, size_t n) {
  typedef typename Io::S S;
  typedef typename Io::C C;
  typedef decltype(Op::fast(C())) St;
  constexpr int PW = 64 * EPT * WPACKS;               // elements per wave
  static_assert(PW <= 65536, "positions are 16-bit");
  __shared__ C q[SPLIT_WAVES * PW];
  const unsigned lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  C* qw = q + wave * PW;
  const size_t wbase = ((size_t)blockIdx.x * SPLIT_WAVES + wave) * PW;
  unsigned nfast = 0, nslow = 0;                       // wave-uniform
  unsigned short pos[WPACKS][EPT];
  bool ok[WPACKS][EPT];
#pragma unroll
  for (int u = 0; u < WPACKS; ++u) {
    C xv[EPT];
    load_lane<Io, EPT, VEC>(x, n, wbase + (size_t)(u * 64 + lane) * EPT, xv, ok[u]);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      bool slow = ok[u][i] && Op::is_slow(xv[i]);
      bool fast = ok[u][i] && !slow;
      unsigned long long mf = __builtin_amdgcn_ballot_w64(fast);
      unsigned long long ms = __builtin_amdgcn_ballot_w64(slow);
      unsigned rf = __builtin_amdgcn_mbcnt_hi((unsigned)(mf >> 32),
                                              __builtin_amdgcn_mbcnt_lo((unsigned)mf, 0u));
      unsigned rs = __builtin_amdgcn_mbcnt_hi((unsigned)(ms >> 32),
                                              __builtin_amdgcn_mbcnt_lo((unsigned)ms, 0u));
      unsigned p = fast ? nfast + rf : PW - 1 - (nslow + rs);
      pos[u][i] = (unsigned short)p;
      if (ok[u][i]) qw[p] = xv[i];
      nfast += (unsigned)__popcll(mf);
      nslow += (unsigned)__popcll(ms);
    }
  }
  wave_lds_sync();
  // dense index d: Cody-Waite elements are d < nfast at position d, the
  // Payne-Hanek ones follow from the back of the region
  for (unsigned d = lane; d < nfast + nslow; d += 64) {
    bool fast = d < nfast;
    unsigned p = fast ? d : PW - 1 - (d - nfast);
    C v = qw[p];
    St st;
    if (fast)
      st = Op::fast(v);
    else
      st = Op::slow(v);
    qw[p] = Op::finish(v, st);
  }
  wave_lds_sync();
#pragma unroll
  for (int u = 0; u < WPACKS; ++u) {
    size_t base = wbase + (size_t)(u * 64 + lane) * EPT;
    if (VEC && base + EPT <= n) {
      Pack<S, EPT> out;
#pragma unroll
      for (int i = 0; i < EPT; ++i) out.v[i] = Io::out(qw[pos[u][i]]);
      store_nt(out, y + base);
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i)
        if (ok[u][i]) y[base + i] = Io::out(qw[pos[u][i]]);
    }
  }
}

// sin and cos of each element in one pass: the Payne-Hanek elements are
// reduced once in the queue (the raw pair and quadrant, the smallest state)
// and mapped to both half-period states afterwards.
template <class Io, class Op, int EPT, bool VEC>
__global__ __launch_bounds__(BLOCK) void k_sincos_split(const typename Io::S* __restrict__ x,
                                                        typename Io::S* __restrict__ ys,
                                                        typename Io::S* __restrict__ yc,
                                                        size_t n) {
  typedef typename Io::S S;
  typedef typename Io::C C;
  typedef decltype(Op::fast(C())) St;
  typedef decltype(Op::slow(C())) Raw;
  __shared__ C q_x[BLOCK * EPT];
  __shared__ unsigned short q_slot[BLOCK * EPT];
  __shared__ Raw q_res[BLOCK * EPT];
  __shared__ unsigned q_cnt[SPLIT_WAVES];
  size_t base = ((size_t)blockIdx.x * BLOCK + threadIdx.x) * EPT;
  C xv[EPT];
  bool ok[EPT];
  load_lane<Io, EPT, VEC>(x, n, base, xv, ok);
  St st[EPT];
  bool slow[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    slow[i] = ok[i] && Op::is_slow(xv[i]);
    st[i] = Op::fast(xv[i]);
  }
  queue_slow<EPT>(xv, slow, q_x, q_slot, q_cnt);
  __syncthreads();
  reduce_queue<EPT>(q_x, q_slot, q_cnt, q_res, [](C v) { return Op::slow(v); });
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i)
    if (slow[i]) st[i] = Op::lift(xv[i], q_res[threadIdx.x * EPT + i]);
  if (VEC && base + EPT <= n) {
    Pack<S, EPT> os, oc;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      os.v[i] = Io::out(Op::finish_sin(xv[i], st[i]));
      oc.v[i] = Io::out(Op::finish_cos(xv[i], st[i]));
    }
    store_nt(os, ys + base);
    store_nt(oc, yc + base);
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      if (ok[i]) {
        ys[base + i] = Io::out(Op::finish_sin(xv[i], st[i]));
        yc[base + i] = Io::out(Op::finish_cos(xv[i], st[i]));
      }
    }
  }
}

// three inputs, two outputs (backward of the binary functions)
template <class Io, class Op, int EPT, bool VEC, int PACKS>
__global__ __launch_bounds__(MAX_BLOCK) void k_ternary2(const typename Io::S* __restrict__ a,
                                                        const typename Io::S* __restrict__ b,
                                                        const typename Io::S* __restrict__ c,
                                                        typename Io::S* __restrict__ y0,
                                                        typename Io::S* __restrict__ y1, size_t n) {
  typedef typename Io::S S;
  typedef typename Io::C C;
  size_t pk0 = (size_t)blockIdx.x * blockDim.x * PACKS + threadIdx.x;
#pragma unroll
  for (int u = 0; u < PACKS; ++u) {
    size_t base = (pk0 + (size_t)u * blockDim.x) * EPT;
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
}


// Elementwise kernels of the integer-operand functions (ldexp, ilogb,
// frexp): one element per lane, grid-stride, any alignment.  T is the
// floating-point type, F a tag with the element function.
constexpr int MAP_BLOCK = 256;
template <class T, class F>
__global__ __launch_bounds__(MAP_BLOCK) void k_ldexp(const T* x, const int* e, T* y, size_t n) {
  size_t stride = (size_t)gridDim.x * MAP_BLOCK;
  for (size_t i = (size_t)blockIdx.x * MAP_BLOCK + threadIdx.x; i < n; i += stride)
    y[i] = F::ldexp(x[i], e[i]);
}
template <class T, class F>
__global__ __launch_bounds__(MAP_BLOCK) void k_ilogb(const T* x, int* e, size_t n) {
  size_t stride = (size_t)gridDim.x * MAP_BLOCK;
  for (size_t i = (size_t)blockIdx.x * MAP_BLOCK + threadIdx.x; i < n; i += stride)
    e[i] = F::ilogb(x[i]);
}
template <class T, class F>
__global__ __launch_bounds__(MAP_BLOCK) void k_remquo(const T* x, const T* y, T* r, int* q,
                                                      size_t n) {
  size_t stride = (size_t)gridDim.x * MAP_BLOCK;
  for (size_t i = (size_t)blockIdx.x * MAP_BLOCK + threadIdx.x; i < n; i += stride) {
    T a = x[i], b = y[i];
    r[i] = F::remquo_rem(a, b);
    q[i] = F::remquo_quo(a, b);
  }
}
template <class T, class F>
__global__ __launch_bounds__(MAP_BLOCK) void k_modf(const T* x, T* f, T* ip, size_t n) {
  size_t stride = (size_t)gridDim.x * MAP_BLOCK;
  for (size_t i = (size_t)blockIdx.x * MAP_BLOCK + threadIdx.x; i < n; i += stride) {
    T v = x[i];
    f[i] = F::modf_frac(v);
    ip[i] = F::modf_int(v);
  }
}
template <class T, class F>
__global__ __launch_bounds__(MAP_BLOCK) void k_fma(const T* a, const T* b, const T* c, T* y,
                                                   size_t n) {
  size_t stride = (size_t)gridDim.x * MAP_BLOCK;
  for (size_t i = (size_t)blockIdx.x * MAP_BLOCK + threadIdx.x; i < n; i += stride)
    y[i] = F::fma(a[i], b[i], c[i]);
}
template <class T, class F, bool ROUND>
__global__ __launch_bounds__(MAP_BLOCK) void k_lrint(const T* x, long long* y, size_t n) {
  size_t stride = (size_t)gridDim.x * MAP_BLOCK;
  for (size_t i = (size_t)blockIdx.x * MAP_BLOCK + threadIdx.x; i < n; i += stride)
    y[i] = ROUND ? F::lround(x[i]) : F::lrint(x[i]);
}
template <class T, class F>
__global__ __launch_bounds__(MAP_BLOCK) void k_frexp(const T* x, T* m, int* e, size_t n) {
  size_t stride = (size_t)gridDim.x * MAP_BLOCK;
  for (size_t i = (size_t)blockIdx.x * MAP_BLOCK + threadIdx.x; i < n; i += stride) {
    T v = x[i];
    m[i] = F::frexp_mant(v);
    e[i] = F::frexp_exp(v);
  }
}

}  // namespace lmh_kernels
