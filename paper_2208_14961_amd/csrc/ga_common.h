// ga_common.h -- block-level helpers shared by libga's kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ga_internal.h"

namespace ga {

// Block-wide minimum of a 64-bit value; the result is valid in thread 0.
__device__ __forceinline__ unsigned long long block_min_u64(
    unsigned long long v) {
  __shared__ unsigned long long s_min[kBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  const int wave = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) s_min[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x / 64); ++w)
      v = s_min[w] < v ? s_min[w] : v;
  }
  return v;
}

// Stop-on-found bookkeeping: a wave whose smallest (key, slot) has key 0
// records generation G as holding a solution.  Rare, so one atomic.
__device__ __forceinline__ void note_zero(RunState* st,
                                          unsigned long long lane_best,
                                          uint32_t G) {
  const bool zero = (lane_best >> 32) == 0;  // invalid lanes carry ~0
  if (__ballot(zero) && (threadIdx.x & 63) == 0) atomicMin(&st->found_gen, G);
}

// Exclusive prefix sum over the block (blockDim.x == kBlock); also returns
// the block total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v,
                                                         uint32_t* total) {
  __shared__ uint32_t s_wave[kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x / 64;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    const uint32_t x = s_wave[w];
    if (w < wave) base += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

static inline uint32_t cdiv(uint64_t a, uint64_t b) {
  return (uint32_t)((a + b - 1) / b);
}

}  // namespace ga
