// ga_select.hip -- selection of the `count` smallest (key, index) of a
// generation: elitism, and the paper's truncation selection (Sec. 3.3).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ga_common.h"
#include "ga_device.h"

namespace ga {

// ---------------------------------------------------------------------------
// Selection of the `count` smallest (key, index) (elitism; the paper's
// truncation, Sec. 3.3): a two-level radix select on 12-bit digits of the
// 24-bit keys, then a stable compaction in index order.
// ---------------------------------------------------------------------------
struct SelArgs {
  uint32_t* pop_a;   // generation g is in the "a" buffers iff g is even
  uint32_t* pop_b;
  uint32_t* keys_a;
  uint32_t* keys_b;
  SelWork* ws;
  RunState* st;
  uint64_t seed;
  uint32_t n, count, mw, paper;
  uint32_t node, max_gen, stop_on_found;
};

// Generation G produced by this launch and whether it runs (see RunState);
// the selection reads generation G - 1.
__device__ __forceinline__ bool sel_generation(const SelArgs& a, uint32_t* G) {
  const uint2 v = *reinterpret_cast<const uint2*>(&a.st->gen_base);
  *G = v.x + a.node + 1;  // v.x = gen_base, v.y = found_gen
  if (*G > a.max_gen) return false;
  if (a.stop_on_found && v.y < *G) return false;
  return true;
}

// Finds the bin holding the target-th element (1-based) of a 4096-bin
// histogram; returns (bin, count before bin).  Clears the histogram.
__device__ void scan_find(uint32_t* hist, uint32_t target, uint32_t* bin_out,
                          uint32_t* before_out) {
  const int per = 4096 / kBlock;  // 16 bins per thread
  uint32_t v[per];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    v[i] = __hip_atomic_load(&hist[threadIdx.x * per + i], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    sum += v[i];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(sum, &total);
#pragma unroll
  for (int i = 0; i < per; ++i) {
    if (run < target && target <= run + v[i]) {
      *bin_out = threadIdx.x * per + i;
      *before_out = run;
    }
    run += v[i];
    hist[threadIdx.x * per + i] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void sel_hist_hi(SelArgs a) {
  uint32_t G;
  if (!sel_generation(a, &G)) return;
  const uint32_t g = G - 1;
  const uint32_t* keys = (g & 1u) ? a.keys_b : a.keys_a;
  __shared__ uint32_t h[4096];
  for (int i = threadIdx.x; i < 4096; i += kBlock) h[i] = 0;
  __syncthreads();
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += gridDim.x * kBlock)
    atomicAdd(&h[(keys[i] >> 12) & 4095u], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < 4096; i += kBlock)
    if (h[i]) atomicAdd(&a.ws->h1[i], h[i]);
  if (last_block(&a.ws->cnt[0])) {
    __shared__ uint32_t s_bin, s_before;
    scan_find(a.ws->h1, a.count, &s_bin, &s_before);
    __syncthreads();
    if (threadIdx.x == 0) {
      a.ws->bucket = s_bin;
      a.ws->below = s_before;
      a.ws->cnt[0] = 0;
    }
  }
}

__global__ __launch_bounds__(kBlock) void sel_hist_lo(SelArgs a) {
  uint32_t G;
  if (!sel_generation(a, &G)) return;
  const uint32_t g = G - 1;
  const uint32_t* keys = (g & 1u) ? a.keys_b : a.keys_a;
  const uint32_t bucket = ld_acq(&a.ws->bucket);
  __shared__ uint32_t h[4096];
  for (int i = threadIdx.x; i < 4096; i += kBlock) h[i] = 0;
  __syncthreads();
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += gridDim.x * kBlock) {
    const uint32_t k = keys[i];
    if ((k >> 12) == bucket) atomicAdd(&h[k & 4095u], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4096; i += kBlock)
    if (h[i]) atomicAdd(&a.ws->h2[i], h[i]);
  if (last_block(&a.ws->cnt[1])) {
    __shared__ uint32_t s_bin, s_before;
    const uint32_t below = ld_acq(&a.ws->below);
    scan_find(a.ws->h2, a.count - below, &s_bin, &s_before);
    __syncthreads();
    if (threadIdx.x == 0) {
      a.ws->T = (bucket << 12) | s_bin;
      a.ws->r = a.count - below - s_before;  // keys equal to T to take
      a.ws->cnt[1] = 0;
    }
  }
}

// Per tile of kSelTile keys: how many are < T and == T; the last block
// turns the per-tile counts into exclusive offsets.
__global__ __launch_bounds__(kBlock) void sel_count(SelArgs a) {
  uint32_t G;
  if (!sel_generation(a, &G)) return;
  const uint32_t g = G - 1;
  const uint32_t* keys = (g & 1u) ? a.keys_b : a.keys_a;
  const uint32_t T = ld_acq(&a.ws->T);
  const uint32_t base = blockIdx.x * kSelTile;
  uint32_t less = 0, eq = 0;
  for (uint32_t i = base + threadIdx.x; i < min(a.n, base + kSelTile);
       i += kBlock) {
    const uint32_t k = keys[i];
    less += k < T;
    eq += k == T;
  }
  uint32_t tl, te;
  block_exclusive_scan(less, &tl);
  block_exclusive_scan(eq, &te);
  if (threadIdx.x == 0) {
    a.ws->blk_less[blockIdx.x] = tl;
    a.ws->blk_eq[blockIdx.x] = te;
  }
  if (last_block(&a.ws->cnt[2])) {
    // exclusive scan over gridDim.x (<= kMaxSelBlocks) tile counts
    const uint32_t nb = gridDim.x;
    const uint32_t per = (nb + kBlock - 1) / kBlock;
    uint32_t sl = 0, se = 0;
    for (uint32_t i = threadIdx.x * per; i < min(nb, (threadIdx.x + 1) * per);
         ++i) {
      sl += __hip_atomic_load(&a.ws->blk_less[i], __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
      se += __hip_atomic_load(&a.ws->blk_eq[i], __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t dummy;
    uint32_t rl = block_exclusive_scan(sl, &dummy);
    uint32_t re = block_exclusive_scan(se, &dummy);
    for (uint32_t i = threadIdx.x * per; i < min(nb, (threadIdx.x + 1) * per);
         ++i) {
      const uint32_t xl = a.ws->blk_less[i], xe = a.ws->blk_eq[i];
      a.ws->blk_less[i] = rl;
      a.ws->blk_eq[i] = re;
      rl += xl;
      re += xe;
    }
    if (threadIdx.x == 0) a.ws->cnt[2] = 0;
  }
}

// Inverse of the keyed Feistel permutation of [0, D) (rounds run backwards,
// cycle-walked into the domain).  For y < D the walk ends within the cycle
// of y; the iteration bound only guarantees termination for any input.
__device__ uint32_t perm_inverse(uint64_t seed, uint32_t G, uint32_t D,
                                 uint32_t y) {
  uint32_t h = 1;
  while ((1ull << (2 * h)) < (uint64_t)D) ++h;
  const uint32_t mask = (1u << h) - 1u;
  const uint64_t limit = 1ull << (2 * h);
  uint32_t x = y;
  for (uint64_t it = 0; it < limit; ++it) {
    uint32_t L = x >> h, R = x & mask;
    for (int r = 7; r >= 0; --r) {
      const U4 u = draw_block(seed, kStreamPerm, G, L, (uint32_t)r >> 2);
      const uint32_t f = u[(uint32_t)r & 3u] & mask;
      const uint32_t nl = R ^ f;
      R = L;
      L = nl;
    }
    x = (L << h) | R;
    if (x < D) break;
  }
  return x;
}

// Stable compaction: the selected individuals, in index order, are copied to
// slots rank (elitism) or pi^-1(rank) (paper mode) of the next generation.
__global__ __launch_bounds__(kBlock) void sel_scatter(SelArgs a) {
  uint32_t G;
  if (!sel_generation(a, &G)) return;
  const uint32_t g = G - 1;
  const bool odd = (g & 1u) != 0;
  const uint32_t* keys = odd ? a.keys_b : a.keys_a;
  const uint32_t* pop = odd ? a.pop_b : a.pop_a;
  uint32_t* pout = odd ? a.pop_a : a.pop_b;
  uint32_t* kout = odd ? a.keys_a : a.keys_b;
  const uint32_t T = ld_acq(&a.ws->T), r = ld_acq(&a.ws->r);
  constexpr int PER = kSelTile / kBlock;  // 8 consecutive keys per thread
  const uint32_t i0 = blockIdx.x * kSelTile + threadIdx.x * PER;
  uint32_t kk[PER];
  uint32_t cl = 0, ce = 0;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    kk[e] = (i0 + e < a.n) ? keys[i0 + e] : 0xffffffffu;
    cl += (i0 + e < a.n) && kk[e] < T;
    ce += (i0 + e < a.n) && kk[e] == T;
  }
  uint32_t dummy;
  uint32_t lb = block_exclusive_scan(cl, &dummy) + a.ws->blk_less[blockIdx.x];
  uint32_t eb = block_exclusive_scan(ce, &dummy) + a.ws->blk_eq[blockIdx.x];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const uint32_t i = i0 + e;
    if (i >= a.n) break;
    const bool less = kk[e] < T, eq = kk[e] == T;
    const bool take = less || (eq && eb < r);
    if (take && lb + min(eb, r) < a.count) {
      const uint32_t rho = lb + min(eb, r);
      const uint32_t slot =
          a.paper ? perm_inverse(a.seed, G, a.count, rho) : rho;
      if (slot < a.count) {
        const uint4* s4 =
            reinterpret_cast<const uint4*>(pop + (size_t)i * a.mw);
        uint4* d4 = reinterpret_cast<uint4*>(pout + (size_t)slot * a.mw);
        for (uint32_t v = 0; v < a.mw / 4; ++v) d4[v] = s4[v];
        kout[slot] = kk[e];
      }
    }
    lb += less;
    eb += eq;
  }
}

hipError_t launch_select(const PopDesc& d, uint32_t count, SelWork* ws,
                         uint32_t node, hipStream_t s) {
  SelArgs a;
  a.pop_a = d.pop_a;
  a.pop_b = d.pop_b;
  a.keys_a = d.keys_a;
  a.keys_b = d.keys_b;
  a.ws = ws;
  a.st = d.state;
  a.seed = d.seed;
  a.n = d.n;
  a.count = count;
  a.mw = d.m * ((d.m + 31) / 32);
  a.paper = d.paper;
  a.node = node;
  a.max_gen = d.max_gen;
  a.stop_on_found = d.stop_on_found;
  const uint32_t gh = std::min<uint32_t>(cdiv(d.n, kBlock * 8), 1024);
  const uint32_t gt = cdiv(d.n, kSelTile);
  hipLaunchKernelGGL(sel_hist_hi, dim3(gh), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(sel_hist_lo, dim3(gh), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(sel_count, dim3(gt), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(sel_scatter, dim3(gt), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace ga
