// ga_elite.hip -- elitism inside ga_run: the next generation's elites from
// a short list instead of the whole population.
//
// Generation G's elites are the e smallest (key, slot) of generation G - 1,
// stored unchanged in slots 0 .. e-1 of G, so every elite precedes every
// child on ties.  With kstar the largest elite key, a child whose key is
// kstar or more is beaten by all e elites, so the e smallest of G are the e
// smallest of the elites and the children below kstar.  The children launch
// of G marks those children in a bitmap over slots; one block then lists
// the marked slots in order after slots 0 .. e-1 (the list is in slot
// order), finds the threshold key T of the e-th smallest by a two-level
// radix select on 12-bit digits (keys are below 2^24), takes the items
// below T and the first items equal to T in slot order, and writes their
// slots in increasing order: the sources of the next elites, with T as the
// next kstar.  The first generation's elites come from every individual,
// chosen by the multi-block selection of ga_select.hip.
#include <hip/hip_runtime.h>

#include "ga_common.h"
#include "ga_scan.h"

namespace ga {

constexpr int kEliteBlock = 1024;

struct EliteArgs {
  const uint32_t* keys_a;  // generation g's keys are in keys_a iff g is even
  const uint32_t* keys_b;
  RunState* st;
  EliteWork* ew;
  uint32_t* mark;          // candidate bitmap over slots, cleared here
  uint32_t* item_slot;     // slots of list entries past the LDS
  uint32_t n, e, node, max_gen, stop_on_found, one_level;
};

// Adds the lanes' bins (those with `valid`) into an LDS histogram: one LDS
// atomic per wave, which serializes lanes on the same bin in the LDS itself.
__device__ __forceinline__ void hist_add(uint32_t* hist, uint32_t bin, bool valid) {
  if (valid) atomicAdd(&hist[bin], 1u);
}

// The same for bins that crowd together (the high digits of the items' keys,
// which all lie below the previous largest elite key, fall into a few bins):
// the wave's most common bins are added with one atomic each, the rest lane
// by lane.  Called by every lane of the wave.
__device__ __forceinline__ void hist_add_crowded(uint32_t* hist, uint32_t bin, bool valid) {
  const uint32_t lane = threadIdx.x & 63u;
  unsigned long long todo = __ballot(valid);
  for (int it = 0; it < 4 && todo; ++it) {
    const int leader = __ffsll((long long)todo) - 1;
    const uint32_t lb = (uint32_t)__builtin_amdgcn_readlane((int)bin, leader);
    const unsigned long long same = __ballot(valid && bin == lb) & todo;
    if ((int)lane == leader) atomicAdd(&hist[lb], (uint32_t)__popcll(same));
    todo &= ~same;
  }
  if ((todo >> lane) & 1ull) atomicAdd(&hist[bin], 1u);
}

// The bin holding the target-th item (1-based) of a 4096-bin LDS histogram,
// and the items before that bin: written by one thread to *bin_out and
// *before_out, read by all after the next barrier.
template <int ID>
__device__ __forceinline__ void find_bin(const uint32_t* hist, uint32_t target,
                                         uint32_t* bin_out, uint32_t* before_out) {
  constexpr int per = 4096 / kEliteBlock;
  uint32_t v[per], sum = 0;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    v[i] = hist[threadIdx.x * per + i];
    sum += v[i];
  }
  uint32_t total;
  uint32_t run = block_scan<kEliteBlock, ID>(sum, &total);
#pragma unroll
  for (int i = 0; i < per; ++i) {
    if (run < target && target <= run + v[i]) {
      *bin_out = threadIdx.x * per + i;
      *before_out = run;
    }
    run += v[i];
  }
}

// Items held in LDS: the keys of up to kLdsItems items, and the slots of
// the candidates among them (items e ..).  Longer lists (and the first
// generation's selection from every individual) read global memory.
constexpr uint32_t kLdsItems = 12288;

// The selection proper over items 0 .. nitems-1 in slot order, read through
// key_at(i) and slot_at(i): the threshold T of the e-th smallest key by a
// two-level radix select (hist_a, hist_b zero on entry), then the stable
// compaction into ew->src.
template <typename KeyAt, typename SlotAt>
__device__ __forceinline__ void select_items(const EliteArgs& a, uint32_t nitems,
                                             uint32_t* hist_a, uint32_t* hist_b,
                                             KeyAt&& key_at, SlotAt&& slot_at) {
  __shared__ uint32_t s_bin, s_before, s_bucket, s_below;
  const uint32_t tid = threadIdx.x, e = a.e;
  uint32_t bucket = 0, below = 0;
  if (!a.one_level) {
    for (uint32_t base = 0; base < nitems; base += kEliteBlock) {
      const uint32_t i = base + tid;
      const bool ok = i < nitems;
      hist_add_crowded(hist_a, ok ? (key_at(i) >> 12) & 4095u : 0u, ok);
    }
    __syncthreads();
    find_bin<1>(hist_a, e, &s_bucket, &s_below);
    __syncthreads();
    bucket = s_bucket;
    below = s_below;
  }
  for (uint32_t base = 0; base < nitems; base += kEliteBlock) {
    const uint32_t i = base + tid;
    const uint32_t k = i < nitems ? key_at(i) : 0u;
    hist_add(hist_b, k & 4095u, i < nitems && (k >> 12) == bucket);
  }
  __syncthreads();
  find_bin<2>(hist_b, e - below, &s_bin, &s_before);
  __syncthreads();
  const uint32_t T = (bucket << 12) | s_bin;
  const uint32_t r = e - below - s_before;  // items equal to T to take
  // stable compaction in slot order: contiguous items per thread
  const uint32_t per = (nitems + kEliteBlock - 1) / kEliteBlock;
  const uint32_t i0 = min(nitems, tid * per), i1 = min(nitems, i0 + per);
  uint32_t less = 0, eq = 0;
  for (uint32_t i = i0; i < i1; ++i) {
    const uint32_t k = key_at(i);
    less += k < T;
    eq += k == T;
  }
  uint2 tot;
  const uint2 off = block_scan2<kEliteBlock, 3>(less, eq, &tot);
  uint32_t lb = off.x, eb = off.y;
  for (uint32_t i = i0; i < i1; ++i) {
    const uint32_t k = key_at(i);
    if (k < T || (k == T && eb < r)) a.ew->src[lb + min(eb, r)] = slot_at(i);
    lb += k < T;
    eb += k == T;
  }
  if (tid == 0) a.ew->kstar = T;
}

// Bitmap words a thread keeps in registers between counting its candidates
// and listing them (populations up to kEliteBlock * 32 * kWordsHeld), and
// elite keys it loads at the start (elite counts up to kEliteBlock *
// kKeysHeld; more are read later).
constexpr uint32_t kWordsHeld = 8;
constexpr uint32_t kKeysHeld = 2;

__device__ __forceinline__ void elite_select_block(const EliteArgs& a) {
  const uint32_t tid = threadIdx.x, e = a.e;
  const uint32_t nw = (a.n + 31u) / 32u;
  const uint32_t per = (nw + kEliteBlock - 1) / kEliteBlock;
  const uint32_t w0 = min(nw, tid * per), w1 = min(nw, w0 + per);
  // Loaded together with the run state: this thread's first bitmap words,
  // and its first elite keys from the key buffer of generation gen_base +
  // node (inside ga_run gen_base is even whenever there are several chunks,
  // so that is the buffer of the node's parity; checked below).
  uint32_t held[kWordsHeld], ekey[kKeysHeld];
  const uint32_t* guess = (a.node & 1u) ? a.keys_b : a.keys_a;
#pragma unroll
  for (uint32_t u = 0; u < kWordsHeld; ++u) held[u] = w0 + u < w1 ? a.mark[w0 + u] : 0u;
#pragma unroll
  for (uint32_t u = 0; u < kKeysHeld; ++u) {
    const uint32_t i = u * kEliteBlock + tid;
    ekey[u] = i < e ? guess[i] : 0u;
  }
  __shared__ uint32_t hist_a[4096], hist_b[4096];
  for (uint32_t i = tid; i < 4096; i += kEliteBlock) {
    hist_a[i] = 0;
    hist_b[i] = 0;
  }
  // the generation whose elites are chosen; it runs only if the children
  // launch before this one made generation Gp - 1 and the run goes on
  const uint2 sv = *reinterpret_cast<const uint2*>(&a.st->gen_base);
  const uint32_t Gp = sv.x + a.node + 1;  // sv.x = gen_base, sv.y = found_gen
  if (Gp > a.max_gen) return;
  if (a.stop_on_found && sv.y < Gp) return;
  const uint32_t g = Gp - 1;
  const uint32_t* keys = (g & 1u) ? a.keys_b : a.keys_a;
  __shared__ uint32_t lkey[kLdsItems], lslot[kLdsItems];
  if (keys != guess) {  // not reached inside ga_run
#pragma unroll
    for (uint32_t u = 0; u < kKeysHeld; ++u) {
      const uint32_t i = u * kEliteBlock + tid;
      ekey[u] = i < e ? keys[i] : 0u;
    }
  }
  // the marked slots (all >= e), in increasing order, become items e ..
  // (slots in LDS, or in item_slot past the LDS), the bitmap is cleared
  uint32_t cnt = 0;
#pragma unroll
  for (uint32_t u = 0; u < kWordsHeld; ++u) cnt += __popc(held[u]);
  for (uint32_t w = w0 + kWordsHeld; w < w1; ++w) cnt += __popc(a.mark[w]);
  uint32_t total;
  uint32_t at = e + block_scan<kEliteBlock, 0>(cnt, &total);
  auto list = [&](uint32_t w, uint32_t bits) {
    while (bits) {
      const uint32_t slot = w * 32u + (uint32_t)(__ffs(bits) - 1);
      if (at < kLdsItems) lslot[at] = slot;
      else a.item_slot[at] = slot;
      ++at;
      bits &= bits - 1u;
    }
  };
#pragma unroll
  for (uint32_t u = 0; u < kWordsHeld; ++u) {
    if (held[u]) {
      a.mark[w0 + u] = 0;
      list(w0 + u, held[u]);
    }
  }
  for (uint32_t w = w0 + kWordsHeld; w < w1; ++w) {
    const uint32_t bits = a.mark[w];
    if (!bits) continue;
    a.mark[w] = 0;
    list(w, bits);
  }
  const uint32_t nitems = e + total;
  if (total == 0) {
    // no child beats the largest elite key: the elites stay, in place, and
    // so does that key
    for (uint32_t i = tid; i < e; i += kEliteBlock) a.ew->src[i] = i;
    return;
  }
  if (nitems <= kLdsItems) {
    // the items' keys into LDS: the elites' from registers (and memory past
    // them), the candidates' gathered eight loads per thread at once
#pragma unroll
    for (uint32_t u = 0; u < kKeysHeld; ++u) {
      const uint32_t i = u * kEliteBlock + tid;
      if (i < e) lkey[i] = ekey[u];
    }
    for (uint32_t i = kKeysHeld * kEliteBlock + tid; i < e; i += kEliteBlock) lkey[i] = keys[i];
    __syncthreads();  // the slot list is complete
    for (uint32_t base = e; base < nitems; base += 8 * kEliteBlock) {
      uint32_t sl[8], k[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t i = base + u * kEliteBlock + tid;
        sl[u] = i < nitems ? lslot[i] : 0u;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) k[u] = keys[sl[u]];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t i = base + u * kEliteBlock + tid;
        if (i < nitems) lkey[i] = k[u];
      }
    }
    __syncthreads();  // the candidates' keys are in
    select_items(a, nitems, hist_a, hist_b, [&](uint32_t i) { return lkey[i]; },
                 [&](uint32_t i) { return i < e ? i : lslot[i]; });
  } else {
    __syncthreads();  // the slot list is complete
    // a long list: its slots past the LDS are in item_slot
    auto slot_at = [&](uint32_t i) {
      return i < e ? i : (i < kLdsItems ? lslot[i] : a.item_slot[i]);
    };
    select_items(a, nitems, hist_a, hist_b, [&](uint32_t i) { return keys[slot_at(i)]; },
                 slot_at);
  }
}

// The arguments of a run's elite selection from its descriptor.
__device__ __host__ __forceinline__ EliteArgs elite_args(const PopDesc& d, uint32_t node,
                                                         uint32_t* item_slot) {
  EliteArgs a;
  a.keys_a = d.keys_a;
  a.keys_b = d.keys_b;
  a.st = d.state;
  a.ew = d.ew;
  a.mark = d.mark;
  a.item_slot = item_slot;
  a.n = d.n;
  a.e = d.elite;
  a.node = node;
  a.max_gen = d.max_gen;
  a.stop_on_found = d.stop_on_found;
  a.one_level = max_key(d.m, d.kind) < 4096 ? 1u : 0u;
  return a;
}

__global__ __launch_bounds__(kEliteBlock) void elite_select_kernel(EliteArgs a) {
  elite_select_block(a);
}

__global__ __launch_bounds__(kEliteBlock) void elite_select_multi_kernel(
    const PopDesc* __restrict__ descs, const uint32_t* __restrict__ runs, uint32_t node) {
  const PopDesc& d = descs[runs[blockIdx.x]];
  elite_select_block(elite_args(d, node, d.eitems));
}

hipError_t launch_elite_select(const PopDesc& d, uint32_t node, uint32_t* item_slot,
                               hipStream_t s) {
  hipLaunchKernelGGL(elite_select_kernel, dim3(1), dim3(kEliteBlock), 0, s,
                     elite_args(d, node, item_slot));
  return hipGetLastError();
}

hipError_t launch_elite_select_multi(const PopDesc* descs_dev, const uint32_t* runs,
                                     uint32_t count, uint32_t node, hipStream_t s) {
  hipLaunchKernelGGL(elite_select_multi_kernel, dim3(count), dim3(kEliteBlock), 0, s, descs_dev,
                     runs, node);
  return hipGetLastError();
}

}  // namespace ga
