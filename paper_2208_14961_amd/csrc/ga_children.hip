// ga_children.hip -- one generation's children: parent selection,
// column-exchange crossover (Sec. 3.4), pair-flip mutation (Sec. 3.5) and
// the child's fitness (Sec. 3.2), one lane per child, fused in one kernel.
// Generation G = state->gen + 1 is produced from generation G - 1; the run
// state's last block closes the generation (best key, stop flag).
#include <hip/hip_runtime.h>

#include "ga_common.h"
#include "ga_device.h"

namespace ga {

// Parents of child pair p: tournaments over generation G-1 (tournament
// mode), or parent slots p and p + N of generation G, already filled by the
// selection kernels (paper mode).  Also returns the child's slot.
struct Parents {
  const uint32_t* A;
  const uint32_t* B;
  uint32_t dst;
};

__device__ __forceinline__ Parents pick_parents(const PopDesc& d, uint32_t G,
                                                uint32_t q, uint32_t MW,
                                                const uint32_t* pin,
                                                const uint32_t* kin,
                                                const uint32_t* pout) {
  const uint32_t p = q >> 1, c = q & 1u;
  Parents r;
  if (d.paper) {
    const uint32_t N = d.n / 4;
    r.A = pout + (size_t)p * MW;
    r.B = pout + (size_t)(p + N) * MW;
    r.dst = (c ? 3u * N : 2u * N) + p;
    return r;
  }
  DrawSeq ds(d.seed, kStreamSelect, G, p);
  uint32_t win[2];
  for (uint32_t s = 0; s < 2; ++s) {
    uint32_t bx = bounded(ds.at(s * d.t), d.n);
    uint32_t bk = kin[bx];
    for (uint32_t k = 1; k < d.t; ++k) {
      const uint32_t x = bounded(ds.at(s * d.t + k), d.n);
      const uint32_t kx = kin[x];
      if (kx < bk || (kx == bk && x < bx)) {
        bx = x;
        bk = kx;
      }
    }
    win[s] = bx;
  }
  r.A = pin + (size_t)win[0] * MW;
  r.B = pin + (size_t)win[1] * MW;
  r.dst = d.elite + q;
  return r;
}

// The four 32-bit words of a lane's Philox block, swapped with lane ^ 1.
__device__ __forceinline__ U4 shfl_xor1(const U4& v) {
  return U4{(uint32_t)__shfl_xor((int)v.x, 1, 64),
            (uint32_t)__shfl_xor((int)v.y, 1, 64),
            (uint32_t)__shfl_xor((int)v.z, 1, 64),
            (uint32_t)__shfl_xor((int)v.w, 1, 64)};
}

// Orders up to 32: the child lives in registers from crossover to store.
// The two children of a pair sit in lanes q and q ^ 1 of one wave: for
// binary tournaments each computes one of the pair's two Philox blocks
// (selection, crossover) and one tournament, and they swap the results.
// All draws come before the dependent loads, so their latency overlaps the
// arithmetic.  Lanes past the last child compute a copy of the last pair
// and store nothing.
template <int M>
__device__ __forceinline__ unsigned long long child(const PopDesc& d,
                                                   uint32_t G, uint32_t q) {
  constexpr uint32_t MW = M;
  const bool odd_in = ((G - 1) & 1u) != 0;
  const uint32_t* pin = odd_in ? d.pop_b : d.pop_a;
  const uint32_t* kin = odd_in ? d.keys_b : d.keys_a;
  uint32_t* pout = odd_in ? d.pop_a : d.pop_b;
  uint32_t* kout = odd_in ? d.keys_a : d.keys_b;
  const bool valid = q < d.nchild;
  const uint32_t npairs = (d.nchild + 1) >> 1;
  const uint32_t p = min(q >> 1, npairs - 1), c = q & 1u;
  const bool binary = !d.paper && d.t == 2;  // uniform over the launch
  U4 xo, sel;
  if (binary) {
    const U4 mine = draw_block(d.seed, c ? kStreamXover : kStreamSelect, G, p, 0);
    const U4 other = shfl_xor1(mine);
    sel = c ? other : mine;
    xo = c ? mine : other;
  } else {
    xo = draw_block(d.seed, kStreamXover, G, p, 0);
    sel = xo;
  }
  const bool mut = (uint64_t)(c ? xo.w : xo.z) < d.mut_thr;
  const uint32_t cut =
      ((uint64_t)xo.x < d.xo_thr) ? 1u + bounded(xo.y, M - 1) : (uint32_t)M;
  // first mutation block, drawn before the loads
  U4 mb0 = U4{0, 0, 0, 0};
  if (mut) mb0 = draw_block(d.seed, kStreamMutate, G, q, 0);
  // parents
  const uint32_t* A;
  const uint32_t* B;
  uint32_t dst;
  if (binary) {
    const uint32_t x0 = bounded(c ? sel.z : sel.x, d.n);
    const uint32_t x1 = bounded(c ? sel.w : sel.y, d.n);
    const uint32_t k0 = kin[x0], k1 = kin[x1];
    const uint32_t w = (k1 < k0 || (k1 == k0 && x1 < x0)) ? x1 : x0;
    const uint32_t wo = (uint32_t)__shfl_xor((int)w, 1, 64);
    A = pin + (size_t)(c ? wo : w) * MW;
    B = pin + (size_t)(c ? w : wo) * MW;
    dst = d.elite + q;
  } else {
    const Parents par = pick_parents(d, G, 2 * p + c, MW, pin, kin, pout);
    A = par.A;
    B = par.B;
    dst = par.dst;
  }
  const uint32_t* first = c ? B : A;
  const uint32_t* second = c ? A : B;
  // mutation (Sec. 3.5): up to four columns by flip masks computed from the
  // parents' words, applied while crossing over; more columns use the
  // general in-register path
  uint32_t mcol[4] = {0, 0, 0, 0}, mmask[4] = {0, 0, 0, 0};
  const bool fast = d.nc <= 4;
  if (mut && fast) {
    DrawSeq ds(d.seed, kStreamMutate, G, q, mb0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if ((uint32_t)k < d.nc) {
        const uint32_t col = 1u + bounded(ds.at(k), M - 1);
        uint32_t v = ((col < cut) ? first : second)[col];
#pragma unroll
        for (int kp = 0; kp < k; ++kp)
          if (mcol[kp] == col) v ^= mmask[kp];
        uint32_t mask = 0;
        for (uint32_t ir = 0; ir < d.nr; ++ir) {
          const uint32_t r1 = bounded(ds.at(d.nc + 2 * ir), M);
          const uint32_t r2 = bounded(ds.at(d.nc + 2 * ir + 1), M);
          const uint32_t x = v ^ mask;
          if (((x >> r1) ^ (x >> r2)) & 1u) mask ^= (1u << r1) | (1u << r2);
        }
        mcol[k] = col;
        mmask[k] = mask;
      }
    }
  }
  Cols<M> cols;
  load_crossed<M>(first, second, cut, cols);
  if (mut) {
    if (fast)
      apply_masks<M>(cols, d.nc, mcol, mmask);
    else
      mutate<M>(cols, d.seed, G, q, d.nc, d.nr);
  }
  const uint32_t key = fitness<M>(cols, d.kind, false, nullptr);
  if (!valid) return ~0ull;
  store_cols<M>(pout + (size_t)dst * MW, cols);
  kout[dst] = key;
  return ((unsigned long long)key << 32) | dst;
}

// Orders 36..64 (two words per column, runtime order): crossover copies the
// columns into the child's slot, mutation edits them there, and the fitness
// reads them back in register tiles.
__device__ __forceinline__ unsigned long long child_w2(const PopDesc& d,
                                                       uint32_t G, uint32_t q) {
  if (q >= d.nchild) return ~0ull;
  const uint32_t M = d.m, MW = 2 * M;
  const bool odd_in = ((G - 1) & 1u) != 0;
  const uint32_t* pin = odd_in ? d.pop_b : d.pop_a;
  const uint32_t* kin = odd_in ? d.keys_b : d.keys_a;
  uint32_t* pout = odd_in ? d.pop_a : d.pop_b;
  uint32_t* kout = odd_in ? d.keys_a : d.keys_b;
  const uint32_t p = q >> 1, c = q & 1u;
  const Parents par = pick_parents(d, G, q, MW, pin, kin, pout);
  const U4 xo = draw_block(d.seed, kStreamXover, G, p, 0);
  const uint32_t cut = ((uint64_t)xo.x < d.xo_thr) ? 1u + bounded(xo.y, M - 1) : M;
  const uint4* f4 = reinterpret_cast<const uint4*>(c ? par.B : par.A);
  const uint4* s4 = reinterpret_cast<const uint4*>(c ? par.A : par.B);
  uint32_t* out = pout + (size_t)par.dst * MW;
  uint4* o4 = reinterpret_cast<uint4*>(out);
  for (uint32_t v = 0; v < M / 2; ++v) {  // 16 bytes = columns 2v, 2v+1
    const uint4 a = f4[v], b = s4[v];
    const bool lo = 2 * v < cut, hi = 2 * v + 1 < cut;
    o4[v] = make_uint4(lo ? a.x : b.x, lo ? a.y : b.y, hi ? a.z : b.z,
                       hi ? a.w : b.w);
  }
  if ((uint64_t)(c ? xo.w : xo.z) < d.mut_thr) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    DrawSeq ds(d.seed, kStreamMutate, G, q);
    for (uint32_t jc = 0; jc < d.nc; ++jc) {
      const uint32_t col = 1u + bounded(ds.at(jc), M - 1);
      uint2* cp = reinterpret_cast<uint2*>(out + 2 * col);
      const uint2 w = *cp;
      uint64_t v = (uint64_t)w.x | ((uint64_t)w.y << 32);
      for (uint32_t ir = 0; ir < d.nr; ++ir) {
        const uint32_t r1 = bounded(ds.at(d.nc + 2 * ir), M);
        const uint32_t r2 = bounded(ds.at(d.nc + 2 * ir + 1), M);
        if (((v >> r1) & 1ull) != ((v >> r2) & 1ull))
          v ^= (1ull << r1) | (1ull << r2);
      }
      *cp = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  const uint32_t key = fitness_w2(out, M, d.kind, false, nullptr);
  kout[par.dst] = key;
  return ((unsigned long long)key << 32) | par.dst;
}

// Generation G of launch `node`, and whether it runs (see RunState).
__device__ __forceinline__ bool generation_of(const PopDesc& d, uint32_t node,
                                              uint32_t* G) {
  const RunState* st = d.state;
  *G = __hip_atomic_load(&st->gen_base, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT) + node + 1;
  if (*G > d.max_gen) return false;
  if (d.stop_on_found &&
      __hip_atomic_load(&st->found_gen, __ATOMIC_RELAXED,
                        __HIP_MEMORY_SCOPE_AGENT) < *G)
    return false;
  return true;
}

// The block's children (one wave); a wave holding a key of 0 records it.
template <typename F>
__device__ __forceinline__ void children_block(const PopDesc& d, uint32_t node,
                                               F&& body) {
  uint32_t G;
  if (!generation_of(d, node, &G)) return;  // uniform over the launch
  const uint32_t q = (blockIdx.x - d.block_begin) * kChildBlock + threadIdx.x;
  note_zero(d.state, body(G, q), G);
}

// One population, order M <= 32, descriptor by value.
template <int M>
__global__ __launch_bounds__(kChildBlock) void children_one_kernel(PopDesc d,
                                                                   uint32_t node) {
  children_block(d, node, [&](uint32_t G, uint32_t q) __attribute__((always_inline)) {
    return child<M>(d, G, q);
  });
}

// One population, order 36..64.
__global__ __launch_bounds__(kChildBlock) void children_one_w2_kernel(
    PopDesc d, uint32_t node) {
  children_block(d, node, [&](uint32_t G, uint32_t q) __attribute__((always_inline)) {
    return child_w2(d, G, q);
  });
}

// Several populations of one order M <= 32 in one launch (block ->
// population through block_pop).  One instantiation per order keeps every
// kernel free of calls: with all orders behind one switch the compiler
// outlines the body into a function longer than the reach of a conditional
// branch, and the long branches it then emits reuse the return-address
// registers, so the function never returns.
template <int M>
__global__ __launch_bounds__(kChildBlock) void children_multi_kernel(
    const PopDesc* __restrict__ descs, const uint32_t* __restrict__ block_pop,
    uint32_t node) {
  const PopDesc d = descs[block_pop[blockIdx.x]];
  children_block(d, node, [&](uint32_t G, uint32_t q) __attribute__((always_inline)) {
    return child<M>(d, G, q);
  });
}

// Several populations of orders 36..64 in one launch.
__global__ __launch_bounds__(kChildBlock) void children_multi_w2_kernel(
    const PopDesc* __restrict__ descs, const uint32_t* __restrict__ block_pop,
    uint32_t node) {
  const PopDesc d = descs[block_pop[blockIdx.x]];
  children_block(d, node, [&](uint32_t G, uint32_t q) __attribute__((always_inline)) {
    return child_w2(d, G, q);
  });
}

hipError_t launch_children(const PopDesc* descs_dev, const uint32_t* block_pop,
                           uint32_t total_blocks, uint32_t m, uint32_t node,
                           hipStream_t s) {
  if (total_blocks == 0) return hipSuccess;
  const dim3 grid(total_blocks), block(kChildBlock);
  switch (m) {
#define GA_MULTI_CASE(MM)                                                    \
  case MM:                                                                   \
    hipLaunchKernelGGL(children_multi_kernel<MM>, grid, block, 0, s,         \
                       descs_dev, block_pop, node);                          \
    break;
    GA_MULTI_CASE(4) GA_MULTI_CASE(8) GA_MULTI_CASE(12) GA_MULTI_CASE(16)
    GA_MULTI_CASE(20) GA_MULTI_CASE(24) GA_MULTI_CASE(28) GA_MULTI_CASE(32)
#undef GA_MULTI_CASE
    default:
      hipLaunchKernelGGL(children_multi_w2_kernel, grid, block, 0, s,
                         descs_dev, block_pop, node);
  }
  return hipGetLastError();
}

hipError_t launch_children_one(const PopDesc& d, uint32_t node, hipStream_t s) {
  if (d.nblocks == 0) return hipSuccess;
  const dim3 grid(d.nblocks), block(kChildBlock);
  switch (d.m) {
#define GA_CH_CASE(MM)                                                      \
  case MM:                                                                  \
    hipLaunchKernelGGL(children_one_kernel<MM>, grid, block, 0, s, d, node);\
    break;
    GA_CH_CASE(4) GA_CH_CASE(8) GA_CH_CASE(12) GA_CH_CASE(16)
    GA_CH_CASE(20) GA_CH_CASE(24) GA_CH_CASE(28) GA_CH_CASE(32)
#undef GA_CH_CASE
    default:
      hipLaunchKernelGGL(children_one_w2_kernel, grid, block, 0, s, d, node);
  }
  return hipGetLastError();
}

}  // namespace ga
