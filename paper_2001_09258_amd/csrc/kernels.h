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

#include "ops.h"

namespace lmh_kernels {
using namespace lmh_ops;

constexpr int BLOCK = 256;          // workgroup of the gathered-trig kernels
constexpr int MAX_BLOCK = 1024;

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
}

// Trigonometric kernel that sorts each workgroup's elements by path.  Every
// element is classified: tiny (the finisher returns x, or 1 for cos,
// without a reduction), Cody-Waite (fast) or Payne-Hanek (slow, including
// non-finite).  A workgroup without slow elements evaluates in place.
// Otherwise the fast elements are appended to an LDS queue from the front
// and the slow ones from the back (one LDS atomic per wave and class:
// ballot, popcount, mbcnt); after a barrier all lanes walk the queue densely
// -- fast items first, then slow -- and write every result into its
// element's slot in LDS (tiny results go there directly); after a second
// barrier each lane stores its own elements with one 16-byte store.  A wave
// thus never runs the Cody-Waite path with most lanes masked off, nor the
// Payne-Hanek path for one large argument.
__device__ __forceinline__ unsigned wave_reserve(bool pred, unsigned* counter) {
  unsigned long long m = __ballot(pred);
  unsigned pre = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                           __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
  unsigned base = 0;
  if (m != 0ull) {
    int leader = __ffsll((long long)m) - 1;
    if (pred && pre == 0u) base = atomicAdd(counter, (unsigned)__popcll(m));
    base = __shfl(base, leader);
  }
  return base + pre;
}

template <class Io, class Op, int EPT, bool VEC>
__global__ __launch_bounds__(BLOCK) void k_unary_split(const typename Io::S* __restrict__ x,
                                                       typename Io::S* __restrict__ y, size_t n) {
  typedef typename Io::S S;
  typedef typename Io::C C;
  typedef decltype(Op::fast(C())) St;
  constexpr int CAP = BLOCK * EPT;
  __shared__ C q_x[CAP];
  __shared__ unsigned short q_slot[CAP];
  __shared__ __align__(16) S q_out[CAP];
  __shared__ unsigned cnt[3];                        // waves with slow elements, queue ends
  if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
  size_t base = ((size_t)blockIdx.x * BLOCK + threadIdx.x) * EPT;
  const bool full = VEC && base + EPT <= n;
  C xv[EPT];
  bool ok[EPT];
  if (full) {
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
  int cls[EPT];                                      // 0 fast, 1 slow, 2 tiny or past the end
  bool any_slow = false;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    cls[i] = !ok[i] || Op::is_tiny(xv[i]) ? 2 : (Op::is_slow(xv[i]) ? 1 : 0);
    any_slow |= cls[i] == 1;
  }
  __syncthreads();                                   // cnt is initialised
  if (__ballot(any_slow) != 0ull && (threadIdx.x & 63u) == 0u) atomicAdd(&cnt[0], 1u);
  __syncthreads();
  if (cnt[0] == 0u) {
    // no Payne-Hanek element in this workgroup: evaluate in place
    if (full) {
      Pack<S, EPT> out;
#pragma unroll
      for (int i = 0; i < EPT; ++i) out.v[i] = Io::out(Op::finish(xv[i], Op::fast(xv[i])));
      store_nt(out, y + base);
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i)
        if (ok[i]) y[base + i] = Io::out(Op::finish(xv[i], Op::fast(xv[i])));
    }
    return;                                          // workgroup-uniform
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const unsigned short slot = (unsigned short)(threadIdx.x * EPT + i);
    unsigned pf = wave_reserve(cls[i] == 0, &cnt[1]);
    unsigned ps = wave_reserve(cls[i] == 1, &cnt[2]);
    if (cls[i] == 0) {
      q_x[pf] = xv[i];
      q_slot[pf] = slot;
    } else if (cls[i] == 1) {
      q_x[CAP - 1 - ps] = xv[i];
      q_slot[CAP - 1 - ps] = slot;
    } else if (ok[i]) {
      q_out[slot] = Io::out(Op::tiny(xv[i]));
    }
  }
  __syncthreads();
  const unsigned nf = cnt[1], ns = cnt[2];
  for (unsigned p = threadIdx.x; p < nf + ns; p += BLOCK) {
    const bool fast = p < nf;
    const unsigned idx = fast ? p : CAP - 1 - (p - nf);
    C xx = q_x[idx];
    St st;
    if (fast)
      st = Op::fast(xx);
    else
      st = Op::slow(xx);
    q_out[q_slot[idx]] = Io::out(Op::finish(xx, st));
  }
  __syncthreads();
  if (full) {
    store_nt(*reinterpret_cast<const Pack<S, EPT>*>(&q_out[threadIdx.x * EPT]), y + base);
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (ok[i]) y[base + i] = q_out[threadIdx.x * EPT + i];
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


}  // namespace lmh_kernels
