// ga_select.hip -- selection of the `count` smallest (key, index) of a
// generation: elitism, and the paper's truncation selection (Sec. 3.3).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ga_common.h"
#include "ga_device.h"

namespace ga {

constexpr uint32_t kFusedTiles = 1024;  // tiles of kSelTile keys

// ---------------------------------------------------------------------------
// Selection of the `count` smallest (key, index) (elitism; the paper's
// truncation, Sec. 3.3): a two-level radix select on 12-bit digits of the
// 24-bit keys, then a stable compaction in index order.  Four launches up to
// kFusedTiles tiles of keys, six above; each kernel boundary orders the
// passes, so no pass needs fences, acquire loads or last-block counters.
// ---------------------------------------------------------------------------
struct SelArgs {
  uint32_t* pop_a;   // generation g is in the "a" buffers iff g is even
  uint32_t* pop_b;
  uint32_t* keys_a;
  uint32_t* keys_b;
  SelWork* ws;
  RunState* st;
  const uint32_t* slots;  // paper mode: slot of each rank for this launch, or null
  uint64_t seed;
  uint32_t n, count, mw, paper;
  uint32_t node, max_gen, stop_on_found;
  uint32_t one_level;  // every key < 4096: the high digit is 0, no first pass
  uint32_t* src_out;    // elitism in ga_run: the scatter writes the selected
  uint32_t* kstar_out;  // sources (src_out[rank]) and T, and copies no rows
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
// histogram; returns (bin, count before bin) through LDS.  With `clear`,
// zeroes the histogram after reading it.
__device__ void scan_find(uint32_t* hist, uint32_t target, bool clear,
                          uint32_t* bin_out, uint32_t* before_out) {
  const int per = 4096 / kBlock;  // 16 bins per thread
  uint32_t v[per];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    v[i] = hist[threadIdx.x * per + i];
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
    if (clear) hist[threadIdx.x * per + i] = 0;
  }
}

// Pass 1: histogram of the high 12 bits of the keys (a block's LDS
// histogram added into h1).  h1 and h2 are zero on entry.
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
}

// Pass 2: every block finds the bucket (high bits) of the count-th key from
// h1, then histograms the low 12 bits of the keys in that bucket into h2.
// When every key of the kind is below 4096 (one_level) the bucket is 0 and
// pass 1 is not launched.
__global__ __launch_bounds__(kBlock) void sel_hist_lo(SelArgs a) {
  uint32_t G;
  if (!sel_generation(a, &G)) return;
  const uint32_t g = G - 1;
  const uint32_t* keys = (g & 1u) ? a.keys_b : a.keys_a;
  __shared__ uint32_t s_bucket, s_below;
  if (a.one_level) {
    if (threadIdx.x == 0) {
      s_bucket = 0;
      s_below = 0;
    }
  } else {
    scan_find(a.ws->h1, a.count, false, &s_bucket, &s_below);
  }
  __shared__ uint32_t h[4096];
  for (int i = threadIdx.x; i < 4096; i += kBlock) h[i] = 0;
  __syncthreads();
  const uint32_t bucket = s_bucket;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ws->bucket = bucket;
    a.ws->below = s_below;
  }
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += gridDim.x * kBlock) {
    const uint32_t k = keys[i];
    if ((k >> 12) == bucket) atomicAdd(&h[k & 4095u], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4096; i += kBlock)
    if (h[i]) atomicAdd(&a.ws->h2[i], h[i]);
}

// One block: the threshold key T and how many keys equal to T to take;
// clears both histograms for the next selection.
__global__ __launch_bounds__(kBlock) void sel_find(SelArgs a) {
  uint32_t G;
  if (!sel_generation(a, &G)) return;
  const uint32_t bucket = a.ws->bucket, below = a.ws->below;
  __shared__ uint32_t s_bin, s_before;
  scan_find(a.ws->h2, a.count - below, true, &s_bin, &s_before);
  for (int i = threadIdx.x; i < 4096; i += kBlock) a.ws->h1[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    a.ws->T = (bucket << 12) | s_bin;
    a.ws->r = a.count - below - s_before;  // keys equal to T to take
  }
}

// Per tile of kSelTile keys: how many are < T and == T.  With `fused`,
// every block first finds T and r from h2 itself (block 0 stores them), in
// place of the one-block sel_find launch.
__global__ __launch_bounds__(kBlock) void sel_count(SelArgs a, uint32_t fused) {
  uint32_t G;
  if (!sel_generation(a, &G)) return;
  const uint32_t g = G - 1;
  const uint32_t* keys = (g & 1u) ? a.keys_b : a.keys_a;
  uint32_t T;
  if (fused) {
    const uint32_t bucket = a.ws->bucket, below = a.ws->below;
    __shared__ uint32_t s_bin, s_before;
    scan_find(a.ws->h2, a.count - below, false, &s_bin, &s_before);
    __syncthreads();
    T = (bucket << 12) | s_bin;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.ws->T = T;
      a.ws->r = a.count - below - s_before;
    }
  } else {
    T = a.ws->T;
  }
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
}

// One block: the per-tile counts become exclusive offsets, in place.
__global__ __launch_bounds__(kBlock) void sel_offsets(SelArgs a, uint32_t nb) {
  uint32_t G;
  if (!sel_generation(a, &G)) return;
  const uint32_t per = (nb + kBlock - 1) / kBlock;
  const uint32_t i0 = min(nb, threadIdx.x * per), i1 = min(nb, i0 + per);
  uint32_t sl = 0, se = 0;
  for (uint32_t i = i0; i < i1; ++i) {
    sl += a.ws->blk_less[i];
    se += a.ws->blk_eq[i];
  }
  uint32_t dummy;
  uint32_t rl = block_exclusive_scan(sl, &dummy);
  uint32_t re = block_exclusive_scan(se, &dummy);
  for (uint32_t i = i0; i < i1; ++i) {
    const uint32_t xl = a.ws->blk_less[i], xe = a.ws->blk_eq[i];
    a.ws->blk_less[i] = rl;
    a.ws->blk_eq[i] = re;
    rl += xl;
    re += xe;
  }
}

// Inverse of the keyed Feistel permutation of [0, D) (rounds run backwards,
// cycle-walked into the domain).  For y < D the walk ends within the cycle
// of y; the iteration bound only guarantees termination for any input.
__device__ __forceinline__ uint32_t feistel_half_bits(uint32_t D) {
  uint32_t h = 1;
  while ((1ull << (2 * h)) < (uint64_t)D) ++h;
  return h;
}
static uint32_t feistel_half_bits_host(uint32_t D) {
  uint32_t h = 1;
  while ((1ull << (2 * h)) < (uint64_t)D) ++h;
  return h;
}

// One inverse evaluation of the eight-round network on 2h bits.
__device__ __forceinline__ uint32_t feistel_inverse(uint64_t seed, uint32_t G,
                                                    uint32_t h, uint32_t x) {
  const uint32_t mask = (1u << h) - 1u;
  uint32_t L = x >> h, R = x & mask;
  for (int r = 7; r >= 0; --r) {
    const U4 u = draw_block(seed, kStreamPerm, G, L, (uint32_t)r >> 2);
    const uint32_t f = u[(uint32_t)r & 3u] & mask;
    const uint32_t nl = R ^ f;
    R = L;
    L = nl;
  }
  return (L << h) | R;
}

__device__ uint32_t perm_inverse(uint64_t seed, uint32_t G, uint32_t D,
                                 uint32_t y) {
  const uint32_t h = feistel_half_bits(D);
  const uint64_t limit = 1ull << (2 * h);
  uint32_t x = y;
  for (uint64_t it = 0; it < limit; ++it) {
    x = feistel_inverse(seed, G, h, x);
    if (x < D) break;
  }
  return x;
}

// The slot pi^-1(rho) of every rank rho < D, for the generations of launches
// 0 .. nodes-1 of a chunk (row `node` for generation gen_base + node + 1);
// with FWD, row r holds instead pi(s) of every parent slot s (the forward
// network).  Each element is a serial cycle walk of eight-round Feistel
// evaluations (about 3.3 on average at 2N = 20,000).  Within one generation
// each round function has only 2^h inputs, so a block first tabulates the
// eight functions of its row in LDS (the two Philox blocks of every input
// value: the same words the network's evaluations draw), and the walks then
// take one table read per round instead of one Philox block.  Element
// (row, e) gets exactly perm_inverse's value; with FWD, the walk of the
// forward network, whose round r maps (L, R) to (R, L xor f_r(R)).  The walks have uneven lengths (up to a dozen evaluations in a wave
// of 64), so each wave owns a pool of its block's elements and a lane that
// ends a walk takes the next element of the pool.
constexpr uint32_t kPermPerBlock = 2048;  // elements of a row per block

template <bool FWD>
__global__ __launch_bounds__(kBlock) void perm_table_kernel(const RunState* st,
                                                            uint64_t seed, uint32_t D,
                                                            uint32_t bpr,
                                                            uint32_t* __restrict__ out) {
  extern __shared__ uint16_t ftab[];  // round r's function at ftab[r * H + v]
  const uint32_t row = blockIdx.x / bpr, part = blockIdx.x % bpr;
  const uint32_t h = feistel_half_bits(D), H = 1u << h, mask = H - 1u;
  const uint32_t G = st->gen_base + row + 1;
  for (uint32_t v = threadIdx.x; v < 2 * H; v += kBlock) {
    const uint32_t in = v >> 1, b = v & 1u;  // rounds 4b .. 4b + 3
    const U4 u = draw_block(seed, kStreamPerm, G, in, b);
    ftab[(4 * b + 0) * H + in] = (uint16_t)(u.x & mask);
    ftab[(4 * b + 1) * H + in] = (uint16_t)(u.y & mask);
    ftab[(4 * b + 2) * H + in] = (uint16_t)(u.z & mask);
    ftab[(4 * b + 3) * H + in] = (uint16_t)(u.w & mask);
  }
  __syncthreads();
  // this block's elements of the row, then this wave's pool of them
  const uint32_t per_block = (D + bpr - 1) / bpr;
  const uint32_t b0 = min(D, part * per_block), b1 = min(D, b0 + per_block);
  constexpr uint32_t kWaves = kBlock / 64;
  const uint32_t wv = threadIdx.x >> 6, per_wave = (b1 - b0 + kWaves - 1) / kWaves;
  const uint32_t begin = min(b1, b0 + wv * per_wave), end = min(b1, begin + per_wave);
  if (begin >= end) return;  // uniform over the wave
  uint32_t* orow = out + (size_t)row * D;
  const uint64_t limit = 1ull << (2 * h);
  const uint32_t lane = threadIdx.x & 63u;
  const unsigned long long below = (1ull << lane) - 1ull;  // lanes before this one
  uint32_t next = begin + 64;  // first element not yet taken (same in every lane)
  uint32_t e = begin + lane;   // this lane's element
  bool busy = e < end;
  uint32_t x = busy ? e : 0u;
  uint64_t it = 0;
  while (__ballot(busy) != 0ull || next < end) {
    if (busy) {
      uint32_t L = x >> h, R = x & mask;
      if (FWD) {
#pragma unroll
        for (uint32_t r = 0; r < 8; ++r) {
          const uint32_t nr = L ^ ftab[r * H + R];
          L = R;
          R = nr;
        }
      } else {
#pragma unroll
        for (int r = 7; r >= 0; --r) {
          const uint32_t nl = R ^ ftab[(uint32_t)r * H + L];
          R = L;
          L = nl;
        }
      }
      x = (L << h) | R;
      if (x < D || ++it == limit) {
        orow[e] = x;
        busy = false;
      }
    }
    const unsigned long long idle = __ballot(!busy);
    if (!busy) {  // take the next element of the pool, in lane order
      const uint32_t mine = next + (uint32_t)__popcll(idle & below);
      if (mine < end) {
        e = mine;
        x = e;
        it = 0;
        busy = true;
      }
    }
    next += (uint32_t)__popcll(idle);
  }
}

hipError_t launch_perm_table(const PopDesc& d, uint32_t count, uint32_t nodes,
                             uint32_t* out, hipStream_t s, bool forward) {
  if (count == 0 || nodes == 0) return hipSuccess;
  const uint32_t bpr = (count + kPermPerBlock - 1) / kPermPerBlock;
  const uint32_t H = 1u << feistel_half_bits_host(count);
  const size_t lds = (size_t)8 * H * sizeof(uint16_t);
  const dim3 grid(nodes * bpr), block(kBlock);
  if (forward)
    hipLaunchKernelGGL(perm_table_kernel<true>, grid, block, lds, s, d.state, d.seed, count, bpr,
                       out);
  else
    hipLaunchKernelGGL(perm_table_kernel<false>, grid, block, lds, s, d.state, d.seed, count,
                       bpr, out);
  return hipGetLastError();
}

// Stable compaction: the selected individuals, in index order, are copied to
// slots rank (elitism) or pi^-1(rank) (paper mode) of the next generation.
// The block first lists its selected (source, slot) pairs in LDS, then
// copies the rows together, each lane issuing its loads before its stores.
// With `fused`, the block sums the per-tile counts before its own tile (in
// place of the one-block sel_offsets launch) and the grid clears h1 and h2.
// `split` blocks share a tile: each lists the tile's selection, and block
// `sub` of them copies rows sub, sub + split, ... of the list; the first
// writes the keys.  Paper mode copies half of every tile, at large orders
// megabytes per generation, which one block per tile would leave to few CUs.
__global__ __launch_bounds__(kBlock) void sel_scatter(SelArgs a, uint32_t fused,
                                                      uint32_t split) {
  uint32_t G;
  if (!sel_generation(a, &G)) return;
  const uint32_t g = G - 1;
  const bool odd = (g & 1u) != 0;
  const uint32_t* keys = odd ? a.keys_b : a.keys_a;
  const uint32_t* pop = odd ? a.pop_b : a.pop_a;
  uint32_t* pout = odd ? a.pop_a : a.pop_b;
  uint32_t* kout = odd ? a.keys_a : a.keys_b;
  const uint32_t T = a.ws->T, r = a.ws->r;
  const uint32_t tile = blockIdx.x / split, sub = blockIdx.x % split;
  uint32_t tile_less, tile_eq;
  if (fused) {
    uint32_t sl = 0, se = 0;
    for (uint32_t b = threadIdx.x; b < tile; b += kBlock) {
      sl += a.ws->blk_less[b];
      se += a.ws->blk_eq[b];
    }
    block_exclusive_scan(sl, &tile_less);
    block_exclusive_scan(se, &tile_eq);
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < 4096; i += gridDim.x * kBlock) {
      a.ws->h1[i] = 0;
      a.ws->h2[i] = 0;
    }
  } else {
    tile_less = a.ws->blk_less[tile];
    tile_eq = a.ws->blk_eq[tile];
  }
  constexpr int PER = kSelTile / kBlock;  // consecutive keys per thread
  const uint32_t i0 = tile * kSelTile + threadIdx.x * PER;
  uint32_t kk[PER];
  uint32_t cl = 0, ce = 0;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    kk[e] = (i0 + e < a.n) ? keys[i0 + e] : 0xffffffffu;
    cl += (i0 + e < a.n) && kk[e] < T;
    ce += (i0 + e < a.n) && kk[e] == T;
  }
  uint32_t dummy;
  uint32_t lb = block_exclusive_scan(cl, &dummy) + tile_less;
  uint32_t eb = block_exclusive_scan(ce, &dummy) + tile_eq;
  // this thread's selected elements: slots in s_dst, sources in s_src
  __shared__ uint32_t s_src[kSelTile], s_dst[kSelTile];
  uint32_t slots[PER];
  uint32_t mine = 0;
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const uint32_t i = i0 + e;
    slots[e] = ~0u;
    if (i < a.n) {
      const bool less = kk[e] < T, eq = kk[e] == T;
      const bool take = less || (eq && eb < r);
      if (take && lb + min(eb, r) < a.count) {
        const uint32_t rho = lb + min(eb, r);
        const uint32_t slot =
            a.paper ? (a.slots ? a.slots[rho] : perm_inverse(a.seed, G, a.count, rho)) : rho;
        if (slot < a.count) {
          slots[e] = slot;
          ++mine;
        }
      }
      lb += less;
      eb += eq;
    }
  }
  uint32_t total;
  uint32_t at = block_exclusive_scan(mine, &total);
  if (a.src_out) {  // the sources of the elites only
#pragma unroll
    for (int e = 0; e < PER; ++e)
      if (slots[e] != ~0u) a.src_out[slots[e]] = i0 + e;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.kstar_out = T;
    return;
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    if (slots[e] != ~0u) {
      s_src[at] = i0 + e;
      s_dst[at] = slots[e];
      if (sub == 0) kout[slots[e]] = kk[e];
      ++at;
    }
  }
  __syncthreads();
  const uint32_t w4 = a.mw / 4, items = total * w4;
  const uint4* src4 = reinterpret_cast<const uint4*>(pop);
  uint4* dst4 = reinterpret_cast<uint4*>(pout);
  // word t of the list: row t / w4, word t % w4 of that row
  auto src_of = [&](uint32_t t) {
    const uint32_t row = t / w4;
    return (size_t)s_src[row] * w4 + (t - row * w4);
  };
  auto dst_of = [&](uint32_t t) {
    const uint32_t row = t / w4;
    return (size_t)s_dst[row] * w4 + (t - row * w4);
  };
  const uint32_t S = split * kBlock;  // this block's words: sub * kBlock + tid + k S
  uint32_t t = sub * kBlock + threadIdx.x;
  for (; t + 3 * S < items; t += 4 * S) {  // four loads, then four stores
    const uint4 v0 = src4[src_of(t)], v1 = src4[src_of(t + S)];
    const uint4 v2 = src4[src_of(t + 2 * S)], v3 = src4[src_of(t + 3 * S)];
    dst4[dst_of(t)] = v0;
    dst4[dst_of(t + S)] = v1;
    dst4[dst_of(t + 2 * S)] = v2;
    dst4[dst_of(t + 3 * S)] = v3;
  }
  for (; t < items; t += S) dst4[dst_of(t)] = src4[src_of(t)];
}

hipError_t launch_select(const PopDesc& d, uint32_t count, SelWork* ws,
                         uint32_t node, const uint32_t* slots, hipStream_t s,
                         uint32_t* src_out, uint32_t* kstar_out) {
  SelArgs a;
  a.src_out = src_out;
  a.kstar_out = kstar_out;
  a.slots = slots;
  a.pop_a = d.pop_a;
  a.pop_b = d.pop_b;
  a.keys_a = d.keys_a;
  a.keys_b = d.keys_b;
  a.ws = ws;
  a.st = d.state;
  a.seed = d.seed;
  a.n = d.n;
  a.count = count;
  a.mw = d.m * col_words(d.m);
  a.paper = d.paper;
  a.node = node;
  a.max_gen = d.max_gen;
  a.stop_on_found = d.stop_on_found;
  a.one_level = max_key(d.m, d.kind) < 4096 ? 1u : 0u;
  const uint32_t gh = std::min<uint32_t>(cdiv(d.n, kSelTile), 1024);
  const uint32_t gt = cdiv(d.n, kSelTile);
  // up to kFusedTiles tiles, the threshold search and the tile offsets are
  // done by every block of the count and scatter launches themselves
  const uint32_t fused = gt <= kFusedTiles;
  if (!a.one_level) hipLaunchKernelGGL(sel_hist_hi, dim3(gh), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(sel_hist_lo, dim3(gh), dim3(kBlock), 0, s, a);
  if (!fused) hipLaunchKernelGGL(sel_find, dim3(1), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(sel_count, dim3(gt), dim3(kBlock), 0, s, a, fused);
  if (!fused) hipLaunchKernelGGL(sel_offsets, dim3(1), dim3(kBlock), 0, s, a, gt);
  // paper mode copies half of every tile: one block per 32 words of a row
  // shares each tile's copy (with the slot table; the inline walk would be
  // repeated by every block of the tile)
  const uint32_t split = (d.paper && slots) ? std::min<uint32_t>(16, cdiv(a.mw, 32)) : 1u;
  hipLaunchKernelGGL(sel_scatter, dim3(gt * split), dim3(kBlock), 0, s, a, fused, split);
  return hipGetLastError();
}

}  // namespace ga
