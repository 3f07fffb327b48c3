// ga_scan.h -- wave and block prefix sums for single-block selection
// kernels (the elite and the paper-mode selections of ga_run).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ga {

// Inclusive prefix sum over the 64 lanes of a wave: shifts by 1, 2, 4 and 8
// within each row of 16 lanes (DPP, lanes shifted in from outside the row
// read 0), then the totals of the rows before (read from lanes 15, 31, 47).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_shr(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  v += dpp_shr<0x111>(v);  // row_shr:1
  v += dpp_shr<0x112>(v);  // row_shr:2
  v += dpp_shr<0x114>(v);  // row_shr:4
  v += dpp_shr<0x118>(v);  // row_shr:8
  const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
  const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
  const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
  const uint32_t row = (threadIdx.x & 63u) >> 4;
  return v + (row > 0 ? r0 : 0u) + (row > 1 ? r1 : 0u) + (row > 2 ? r2 : 0u);
}

// The sum over the wave, in every lane.
__device__ __forceinline__ uint32_t wave_total(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_inclusive_scan(v), 63);
}

// Exclusive prefix sums of two values over a block of NT threads, and their
// totals.  Each call site passes its own ID, so the wave totals of one call
// are never overwritten by a later one: one barrier per call.
template <int NT, int ID>
__device__ __forceinline__ uint2 block_scan2(uint32_t a, uint32_t b, uint2* total) {
  constexpr int kWaves = NT / 64;
  __shared__ uint2 s_wave[kWaves];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t ia = wave_inclusive_scan(a), ib = wave_inclusive_scan(b);
  if (lane == 63) s_wave[wave] = make_uint2(ia, ib);
  __syncthreads();
  uint2 base = make_uint2(0, 0), tot = make_uint2(0, 0);
#pragma unroll
  for (uint32_t w = 0; w < kWaves; ++w) {
    const uint2 x = s_wave[w];
    if (w < wave) {
      base.x += x.x;
      base.y += x.y;
    }
    tot.x += x.x;
    tot.y += x.y;
  }
  *total = tot;
  return make_uint2(base.x + ia - a, base.y + ib - b);
}
template <int NT, int ID>
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* total) {
  uint2 t;
  const uint2 r = block_scan2<NT, ID>(v, 0u, &t);
  *total = t.x;
  return r.x;
}

}  // namespace ga
