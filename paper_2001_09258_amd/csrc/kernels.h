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

// Trigonometric kernel with the Payne-Hanek lanes gathered.  Each lane
// classifies its elements; the Cody-Waite ones are reduced in place, the
// others are appended to a workgroup queue in LDS (one LDS atomic per wave:
// ballot, popcount, mbcnt) and reduced densely by all lanes after a barrier,
// so a wave that holds a few large arguments no longer pays the whole
// Payne-Hanek path.  The reduced states come back through LDS and every lane
// finishes its own elements.
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
  __shared__ C q_x[BLOCK * EPT];
  __shared__ unsigned short q_slot[BLOCK * EPT];
  __shared__ St q_res[BLOCK * EPT];
  __shared__ unsigned q_cnt;
  if (threadIdx.x == 0) q_cnt = 0;
  size_t base = ((size_t)blockIdx.x * BLOCK + threadIdx.x) * EPT;
  C xv[EPT];
  bool ok[EPT];
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
  __syncthreads();                                   // q_cnt is initialised
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
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    unsigned pos = wave_reserve(slow[i], &q_cnt);
    if (slow[i]) {
      q_x[pos] = xv[i];
      q_slot[pos] = (unsigned short)(threadIdx.x * EPT + i);
    }
  }
  __syncthreads();
  const unsigned cnt = q_cnt;
  for (unsigned p = threadIdx.x; p < cnt; p += BLOCK) q_res[q_slot[p]] = Op::slow(q_x[p]);
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
