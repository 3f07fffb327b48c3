// ga_paper.hip -- the paper's truncation selection (Sec. 3.3) inside ga_run
// for populations up to kPaperTileMaxN.
//
// The 2N smallest (key, index) of generation G - 1 (of 4N), listed in index
// order, are sel[0 .. 2N-1]; parent slot s of G receives sel[pi(s)], pi the
// keyed permutation of the generation.  With T the 2N-th smallest key, sel
// holds every key below T and, in index order, the first r keys equal to T
// (r = 2N - #keys below T).
//
// Two launches over tiles of kPaperTile keys (one block of 1024 threads, four
// keys a thread):
//  * count: each tile counts its keys at top - d for d < kPaperBins (LDS
//    bins) and below that window, and writes for each d its keys at distance
//    d or more (a suffix sum) and its keys below; top is the previous
//    selection's T.  T never increases from one generation to the next (the
//    2N parents of a generation carry keys <= the T that selected them), so
//    T lies in [0, top], and in practice within the window.
//  * list: every tile adds the tiles' suffix sums (thread t takes d = t: the
//    count of keys <= top - d without a scan), finds T and r and the counts of
//    selected keys below T and equal to T in the tiles before it (two words
//    of each), ranks its own selected keys with a block scan, and writes
//    sel[rho] = index for rank rho.  Without a previous T, top is the
//    largest key of the fitness kind; if T lies below the window, each tile
//    finds it by counting all keys (the slow path).
// The children launch then reads parent slot s's individual as sel[pi(s)],
// pi(s) from the chunk's forward table.  Each launch reads what the one before
// wrote on other XCDs: its loads are issued together, since a dependent chain
// costs a memory round trip a link.  T alternates between two words (the
// list launch writes generation G's while its tiles read G - 1's), and the
// search for T is repeated in every tile rather than done by the last tile
// of the count launch: a device-wide fence there (an L2 write-back) cost more
// than the repeated work.
#include <hip/hip_runtime.h>

#include "ga_common.h"
#include "ga_scan.h"

namespace ga {

constexpr int kPaperBlock = 1024;
static_assert(kPaperTile == 4 * kPaperBlock, "four keys a thread");
static_assert(kPaperBins == kPaperBlock, "one window bin a thread");

struct PaperArgs {
  const uint32_t* keys_a;  // generation g's keys are in keys_a iff g is even
  const uint32_t* keys_b;
  RunState* st;
  PaperWork* pw;
  uint32_t* sel;           // 2N: the selected indices in index order
  uint32_t n, D, node, max_gen, stop_on_found, key_bound, ntiles;
};

// The generation whose parents this launch selects, and whether it runs.
__device__ __forceinline__ bool paper_generation(const PaperArgs& a, uint32_t* G) {
  const uint2 v = *reinterpret_cast<const uint2*>(&a.st->gen_base);
  *G = v.x + a.node + 1;
  if (*G > a.max_gen) return false;
  if (a.stop_on_found && v.y < *G) return false;
  return true;
}

// The four keys of a thread, from index i0 (past n: ~0, never selected).
__device__ __forceinline__ uint4 tile_keys(const uint32_t* keys, uint32_t n, uint32_t i0) {
  if (i0 + 3 < n && (reinterpret_cast<uintptr_t>(keys) & 15u) == 0)
    return *reinterpret_cast<const uint4*>(keys + i0);
  uint4 v;
  v.x = i0 < n ? keys[i0] : ~0u;
  v.y = i0 + 1 < n ? keys[i0 + 1] : ~0u;
  v.z = i0 + 2 < n ? keys[i0 + 2] : ~0u;
  v.w = i0 + 3 < n ? keys[i0 + 3] : ~0u;
  return v;
}

// The block's sum of v (one barrier; the two buffers alternate, so a call's
// writes never meet the previous call's reads).
__device__ __forceinline__ uint32_t paper_block_sum(uint32_t v, uint32_t (*buf)[kPaperBlock / 64],
                                                    uint32_t& which) {
  const uint32_t t = wave_total(v);
  if ((threadIdx.x & 63u) == 0) buf[which][threadIdx.x >> 6] = t;
  __syncthreads();
  uint32_t s = 0;
#pragma unroll
  for (int w = 0; w < kPaperBlock / 64; ++w) s += buf[which][w];
  which ^= 1u;
  return s;
}

// The arguments of a run's selection from its descriptor.
__device__ __host__ __forceinline__ PaperArgs paper_args(const PopDesc& d, uint32_t node,
                                                         uint32_t* sel) {
  PaperArgs a;
  a.keys_a = d.keys_a;
  a.keys_b = d.keys_b;
  a.st = d.state;
  a.pw = d.pw;
  a.sel = sel;
  a.n = d.n;
  a.D = d.n / 2;
  a.node = node;
  a.max_gen = d.max_gen;
  a.stop_on_found = d.stop_on_found;
  a.key_bound = (uint32_t)max_key(d.m, d.kind);
  a.ntiles = (d.n + kPaperTile - 1) / kPaperTile;
  return a;
}

// Tile b of the count launch.
__device__ __forceinline__ void paper_count_tile(const PaperArgs& a, uint32_t b) {
  uint32_t G;
  if (!paper_generation(a, &G)) return;  // uniform over the block
  const uint32_t* keys = ((G - 1) & 1u) ? a.keys_b : a.keys_a;
  PaperWork* pw = a.pw;
  const uint32_t prev = pw->T[(G - 1) & 1u];
  const uint32_t top = prev == ~0u ? a.key_bound : prev;
  const uint32_t tid = threadIdx.x;
  __shared__ uint32_t h[kPaperBins];
  __shared__ uint32_t red[2][kPaperBlock / 64];
  h[tid] = 0;
  __syncthreads();
  const uint4 k4 = tile_keys(keys, a.n, b * kPaperTile + 4 * tid);
  uint32_t below = 0;
  auto add = [&](uint32_t k) {
    if (k <= top) {
      const uint32_t d = top - k;
      if (d < kPaperBins) atomicAdd(&h[d], 1u);
      else ++below;
    }
  };
  add(k4.x);
  add(k4.y);
  add(k4.z);
  add(k4.w);
  uint32_t which = 0;
  const uint32_t tile_below = paper_block_sum(below, red, which);  // its barrier ends the adds
  // thread t: d = kPaperBins - 1 - t, so the inclusive prefix over threads is
  // the tile's keys at distance d or more
  const uint32_t d = kPaperBins - 1 - tid, hd = h[d];
  uint32_t total;
  const uint32_t cum = block_scan<kPaperBlock, 3>(hd, &total) + hd;
  pw->hist[b][d] = cum;
  if (tid == 0) pw->hist[b][kPaperBins] = tile_below;
}

// Tile b of the list launch.
__device__ __forceinline__ void paper_list_tile(const PaperArgs& a, uint32_t b) {
  uint32_t G;
  if (!paper_generation(a, &G)) return;
  const uint32_t* keys = ((G - 1) & 1u) ? a.keys_b : a.keys_a;
  PaperWork* pw = a.pw;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, D = a.D;
  const uint32_t i0 = b * kPaperTile + 4 * tid;
  const uint32_t prev = pw->T[(G - 1) & 1u];
  const uint32_t top = prev == ~0u ? a.key_bound : prev;
  // every load at once: this tile's keys, every tile's suffix sum at d = t,
  // and every tile's count below the window (the same words in every thread)
  const uint4 k4 = tile_keys(keys, a.n, i0);
  const uint32_t d = tid;
  uint32_t hv[kPaperMaxTiles], S = 0, below = 0;
#pragma unroll
  for (uint32_t t = 0; t < kPaperMaxTiles; ++t) {
    hv[t] = t < a.ntiles ? pw->hist[t][d] : 0u;
    below += t < a.ntiles ? pw->hist[t][kPaperBins] : 0u;
  }
  const uint32_t own_below = tid < a.ntiles ? pw->hist[tid][kPaperBins] : 0u;
#pragma unroll
  for (uint32_t t = 0; t < kPaperMaxTiles; ++t) S += hv[t];
  __shared__ uint32_t red[2][kPaperBlock / 64];
  __shared__ uint32_t s_le[kPaperBins];
  __shared__ uint32_t s_c[2][kPaperMaxTiles];  // each tile's suffix sums at d* and d* + 1
  __shared__ uint32_t s_below[kPaperMaxTiles];
  if (tid < kPaperMaxTiles) s_below[tid] = own_below;
  __shared__ uint32_t s_T, s_r, s_ds, s_found, s_less0, s_eq0;
  uint32_t which = 0;
  const uint32_t le = below + S;  // keys <= top - d
  s_le[d] = le;
  if (tid == 0) s_found = 0;
  __syncthreads();
  const uint32_t lt = d + 1 < kPaperBins ? s_le[d + 1] : below;  // keys < top - d
  if (tid < kPaperMaxTiles) s_c[1][tid] = 0;  // d* + 1 past the window
  if (below < D && le >= D && lt < D) {  // at most one thread: T = top - d
    s_T = top - d;
    s_r = D - lt;
    s_ds = d;
    s_found = 1;
#pragma unroll
    for (uint32_t t = 0; t < kPaperMaxTiles; ++t) s_c[0][t] = hv[t];
  }
  __syncthreads();
  if (s_found) {
    // the tiles before this one: keys below the window or at distance > d*,
    // and keys at d*, from the suffix sums the threads of d* and d* + 1 hold
    if (d == s_ds + 1) {
#pragma unroll
      for (uint32_t t = 0; t < kPaperMaxTiles; ++t) s_c[1][t] = hv[t];
    }
    __syncthreads();
    if (wave == 0) {
      uint32_t l = 0, e = 0;
      if (lane < b) {
        l = s_below[lane] + s_c[1][lane];
        e = s_c[0][lane] - s_c[1][lane];
      }
      l = wave_total(l);
      e = wave_total(e);
      if (lane == 0) {
        s_less0 = l;
        s_eq0 = e;
      }
    }
  } else {
    // slow path: T below the window (or fewer than 2N keys at or below top):
    // count all keys, bisecting [0, hi] with count(<= hi) >= 2N
    uint32_t lo = 0, hi = below >= D ? top - kPaperBins : a.key_bound;
    auto count = [&](uint32_t x, uint32_t end) {
      uint32_t c = 0;
      for (uint32_t j0 = 4 * tid; j0 < end; j0 += kPaperTile) {
        const uint4 k = tile_keys(keys, a.n, j0);
        c += (k.x <= x ? 1u : 0u) + (k.y <= x ? 1u : 0u) + (k.z <= x ? 1u : 0u) +
             (k.w <= x ? 1u : 0u);
      }
      return paper_block_sum(c, red, which);
    };
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo) / 2;
      if (count(mid, a.n) >= D) hi = mid;
      else lo = mid + 1;
    }
    const uint32_t T = lo;
    const uint32_t nlt = T > 0 ? count(T - 1, a.n) : 0u;
    // the tiles before this one, by counting their keys
    const uint32_t l0 = T > 0 ? count(T - 1, b * kPaperTile) : 0u;
    const uint32_t le0 = count(T, b * kPaperTile);
    if (tid == 0) {
      s_T = T;
      s_r = D - nlt;
      s_less0 = l0;
      s_eq0 = le0 - l0;
    }
  }
  __syncthreads();
  const uint32_t T = s_T, r = s_r;
  if (b == 0 && tid == 0) pw->T[G & 1u] = T;
  const uint32_t k[4] = {k4.x, k4.y, k4.z, k4.w};
  uint32_t lc = 0, ec = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    lc += k[j] < T ? 1u : 0u;
    ec += k[j] == T ? 1u : 0u;
  }
  uint2 tot;
  const uint2 ex = block_scan2<kPaperBlock, 1>(lc, ec, &tot);
  uint32_t lb = s_less0 + ex.x, eb = s_eq0 + ex.y;  // keys below T / equal to T before
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool lt = k[j] < T, eq = k[j] == T;
    if (lt || (eq && eb < r)) a.sel[lb + min(eb, r)] = i0 + j;
    lb += lt ? 1u : 0u;
    eb += eq ? 1u : 0u;
  }
}

__global__ __launch_bounds__(kPaperBlock) void paper_count_kernel(PaperArgs a) {
  paper_count_tile(a, blockIdx.x);
}
__global__ __launch_bounds__(kPaperBlock) void paper_list_kernel(PaperArgs a) {
  paper_list_tile(a, blockIdx.x);
}

// Several runs: block b takes tile (e & 15) of run descs[e >> 4], e = tiles[b].
__global__ __launch_bounds__(kPaperBlock) void paper_count_multi_kernel(
    const PopDesc* __restrict__ descs, const uint32_t* __restrict__ tiles, uint32_t node) {
  const uint32_t e = tiles[blockIdx.x];
  const PopDesc& d = descs[e >> 4];
  paper_count_tile(paper_args(d, node, d.psel), e & 15u);
}
__global__ __launch_bounds__(kPaperBlock) void paper_list_multi_kernel(
    const PopDesc* __restrict__ descs, const uint32_t* __restrict__ tiles, uint32_t node) {
  const uint32_t e = tiles[blockIdx.x];
  const PopDesc& d = descs[e >> 4];
  paper_list_tile(paper_args(d, node, d.psel), e & 15u);
}

hipError_t launch_paper_select(const PopDesc& d, uint32_t node, uint32_t* sel, hipStream_t s) {
  if (d.n > kPaperTileMaxN) return hipErrorInvalidValue;
  const PaperArgs a = paper_args(d, node, sel);
  hipLaunchKernelGGL(paper_count_kernel, dim3(a.ntiles), dim3(kPaperBlock), 0, s, a);
  hipLaunchKernelGGL(paper_list_kernel, dim3(a.ntiles), dim3(kPaperBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_paper_select_multi(const PopDesc* descs_dev, const uint32_t* tiles,
                                     uint32_t nblocks, uint32_t node, hipStream_t s) {
  hipLaunchKernelGGL(paper_count_multi_kernel, dim3(nblocks), dim3(kPaperBlock), 0, s, descs_dev,
                     tiles, node);
  hipLaunchKernelGGL(paper_list_multi_kernel, dim3(nblocks), dim3(kPaperBlock), 0, s, descs_dev,
                     tiles, node);
  return hipGetLastError();
}

}  // namespace ga
