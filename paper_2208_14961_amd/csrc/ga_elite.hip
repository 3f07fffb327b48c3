// ga_elite.hip -- elitism in ga_run, batched and served runs: the next
// generation's elites from short candidate lists instead of the whole
// population.
//
// Generation G's elites are the e smallest (key, slot) of generation G - 1,
// stored unchanged in slots 0 .. e-1 of G, so every elite precedes every
// child on ties.  With kstar the largest elite key, a child whose key is
// kstar or more is beaten by all e elites, so the e smallest of G are the e
// smallest of the elites and the children below kstar.  The children launch
// of G appends those children, as (slot, key), to kEliteLists lists.  One
// block then puts them in slot order after the elites (a bitmap of the
// listed slots and its prefix counts give each its rank), finds the
// threshold key T of the e-th smallest item (every item is at most kstar:
// one histogram of the 4096 keys up to kstar, or, when T lies below them, a
// two-level radix select on 12-bit digits of keys below 2^24), takes the
// items below T and the first items equal to T in slot order, and writes
// their slots in increasing order: the sources of the next elites, with T
// as the next kstar.  The first generation's elites come from every
// individual, chosen by the multi-block selection of ga_select.hip.
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
  uint32_t* count;         // the kEliteLists candidate counts, cleared here
  const uint2* list;       // the candidate lists, list j from entry j * cap
  uint32_t* scratch;       // slot bitmap, prefix counts, item keys and slots
                           // for cases too large for the LDS
  uint32_t cap, n, e, node, max_gen, stop_on_found, one_level;
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

// Items (the elites, then the listed children in slot order) whose keys and
// slots are held in LDS, and slot bitmap words held in LDS (populations up
// to 32 * kLdsWords); larger cases use the scratch area in global memory.
constexpr uint32_t kLdsItems = 10240;
constexpr uint32_t kLdsWords = 8192;

// The selection proper over items 0 .. nitems-1 in slot order, read through
// key_at(i) and slot_at(i), every key at most kprev (the largest elite key,
// which every listed child is below): the threshold T of the e-th smallest
// key, then the stable compaction into ew->src.  T comes from one histogram
// of the keys in the window kprev - 4095 .. kprev when fewer than e keys lie
// below it, else from a two-level radix select on 12-bit digits.  hist_a and
// hist_b are zero on entry, and *s_low (items below the window) too.
template <typename KeyAt, typename SlotAt>
__device__ __forceinline__ void select_items(const EliteArgs& a, uint32_t nitems,
                                             uint32_t kprev, uint32_t* hist_a,
                                             uint32_t* hist_b, uint32_t* s_low,
                                             KeyAt&& key_at, SlotAt&& slot_at) {
  __shared__ uint32_t s_bin, s_before, s_bucket, s_below;
  const uint32_t tid = threadIdx.x, e = a.e;
  const uint32_t lo = kprev > 4095u ? kprev - 4095u : 0u;
  uint32_t low = 0;
  for (uint32_t base = 0; base < nitems; base += kEliteBlock) {
    const uint32_t i = base + tid;
    const uint32_t k = i < nitems ? key_at(i) : lo;
    const bool in = i < nitems && k >= lo;
    low += i < nitems && k < lo;
    hist_add(hist_a, min(k - lo, 4095u), in);
  }
  low = wave_total(low);
  if ((tid & 63u) == 0 && low) atomicAdd(s_low, low);
  __syncthreads();
  uint32_t T, r;
  if (*s_low < e) {  // the e-th smallest key is in the window
    const uint32_t B = *s_low;
    find_bin<1>(hist_a, e - B, &s_bin, &s_before);
    __syncthreads();
    T = lo + s_bin;
    r = e - B - s_before;  // items equal to T to take
  } else {
    for (uint32_t i = tid; i < 4096; i += kEliteBlock) hist_a[i] = 0;
    __syncthreads();
    uint32_t bucket = 0, below = 0;
    if (!a.one_level) {
      for (uint32_t base = 0; base < nitems; base += kEliteBlock) {
        const uint32_t i = base + tid;
        const bool ok = i < nitems;
        hist_add_crowded(hist_a, ok ? (key_at(i) >> 12) & 4095u : 0u, ok);
      }
      __syncthreads();
      find_bin<2>(hist_a, e, &s_bucket, &s_below);
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
    find_bin<5>(hist_b, e - below, &s_bin, &s_before);
    __syncthreads();
    T = (bucket << 12) | s_bin;
    r = e - below - s_before;
  }
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

// List entries a thread holds: threads 4j .. 4j+3 take list j's entries
// q, q + 4, ... (q = thread & 3), the first kHeld each in registers (read
// at the start, with the run state); longer lists are read in a loop.
constexpr uint32_t kHeld = 10;
static_assert(kEliteBlock == 4 * kEliteLists, "four threads per candidate list");

// (The bitmap is read with atomic loads: in global memory its words were
// set by atomics, which bypass the compute unit's cache.)
__device__ __forceinline__ uint32_t bits_at(uint32_t* bits, uint32_t w) {
  return __hip_atomic_load(&bits[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The listed children become items e .. e + total - 1 in slot order: each
// listed slot is set in a bitmap (nw words, zero on entry), the prefix
// counts of its words (wpre) give each slot's rank among them, and the
// child of rank r goes to ikey[e + r], islot[e + r].  (lst, q, c) name this
// thread's share of the lists; en holds its first kHeld entries.
__device__ __forceinline__ void order_children(const EliteArgs& a, uint32_t lst, uint32_t q,
                                               uint32_t c, const uint2 (&en)[kHeld],
                                               uint32_t nw, uint32_t* bits, uint32_t* wpre,
                                               uint32_t* ikey, uint32_t* islot) {
  const uint32_t tid = threadIdx.x;
  const uint2* mine = a.list + (size_t)lst * a.cap;
#pragma unroll
  for (uint32_t k = 0; k < kHeld; ++k)
    if (q + 4 * k < c) atomicOr(&bits[en[k].x >> 5], 1u << (en[k].x & 31u));
  for (uint32_t i = q + 4 * kHeld; i < c; i += 4) {
    const uint32_t slot = mine[i].x;
    atomicOr(&bits[slot >> 5], 1u << (slot & 31u));
  }
  __syncthreads();
  // thread t's words: t * per .. (t + 1) * per - 1
  const uint32_t per = (nw + kEliteBlock - 1) / kEliteBlock;
  const uint32_t w0 = min(nw, tid * per), w1 = min(nw, w0 + per);
  uint32_t cnt = 0;
  for (uint32_t w = w0; w < w1; ++w) cnt += __popc(bits_at(bits, w));
  uint32_t listed;
  uint32_t at = block_scan<kEliteBlock, 4>(cnt, &listed);
  for (uint32_t w = w0; w < w1; ++w) {
    wpre[w] = at;
    at += __popc(bits_at(bits, w));
  }
  __syncthreads();
  auto place = [&](const uint2 x) {
    const uint32_t w = x.x >> 5;
    const uint32_t rank = wpre[w] + __popc(bits_at(bits, w) & ((1u << (x.x & 31u)) - 1u));
    ikey[a.e + rank] = x.y;
    islot[a.e + rank] = x.x;
  };
#pragma unroll
  for (uint32_t k = 0; k < kHeld; ++k)
    if (q + 4 * k < c) place(en[k]);
  for (uint32_t i = q + 4 * kHeld; i < c; i += 4) place(mine[i]);
}

// Elite keys a thread loads at the start (elite counts up to kEliteBlock *
// kKeysHeld; more are read later).
constexpr uint32_t kKeysHeld = 2;

__device__ __forceinline__ void elite_select_block(const EliteArgs& a) {
  const uint32_t tid = threadIdx.x, e = a.e;
  const uint32_t nw = (a.n + 31u) / 32u;
  // Loaded together with the run state: this thread's share of the lists,
  // the largest elite key, and this thread's first elite keys from the key
  // buffer of generation gen_base + node (inside ga_run gen_base is even
  // whenever there are several chunks, so that is the buffer of the node's
  // parity; checked below).
  const uint32_t lst = tid >> 2, q = tid & 3u;
  const uint32_t c = min(a.count[lst], a.cap);
  uint2 en[kHeld];
#pragma unroll
  for (uint32_t k = 0; k < kHeld; ++k)
    en[k] = q + 4 * k < c ? a.list[(size_t)lst * a.cap + q + 4 * k] : make_uint2(0, 0);
  const uint32_t kprev = a.ew->kstar;
  uint32_t ekey[kKeysHeld];
  const uint32_t* guess = (a.node & 1u) ? a.keys_b : a.keys_a;
#pragma unroll
  for (uint32_t u = 0; u < kKeysHeld; ++u) {
    const uint32_t i = u * kEliteBlock + tid;
    ekey[u] = i < e ? guess[i] : 0u;
  }
  // the histograms of the selection, which first hold the prefix counts of
  // the slot bitmap
  __shared__ uint32_t hist[2 * 4096], lbits[kLdsWords], s_low;
  for (uint32_t i = tid; i < 2 * 4096; i += kEliteBlock) hist[i] = 0;
  if (nw <= kLdsWords)
    for (uint32_t i = tid; i < nw; i += kEliteBlock) lbits[i] = 0;
  if (tid == 0) s_low = 0;
  // the generation whose elites are chosen; it runs only if the children
  // launch before this one made generation Gp - 1 and the run goes on
  const uint2 sv = *reinterpret_cast<const uint2*>(&a.st->gen_base);
  const uint32_t Gp = sv.x + a.node + 1;  // sv.x = gen_base, sv.y = found_gen
  if (Gp > a.max_gen) return;
  if (a.stop_on_found && sv.y < Gp) return;
  const uint32_t g = Gp - 1;
  const uint32_t* keys = (g & 1u) ? a.keys_b : a.keys_a;
  if (keys != guess) {  // not reached inside ga_run
#pragma unroll
    for (uint32_t u = 0; u < kKeysHeld; ++u) {
      const uint32_t i = u * kEliteBlock + tid;
      ekey[u] = i < e ? keys[i] : 0u;
    }
  }
  // the lists' counts start from zero for the next children launch (which
  // runs after this one)
  if (q == 0 && c) a.count[lst] = 0;
  uint32_t total;
  (void)block_scan<kEliteBlock, 0>(q == 0 ? c : 0u, &total);
  if (total == 0) {
    // no child beats the largest elite key: the elites stay, in place, and
    // so does that key
    for (uint32_t i = tid; i < e; i += kEliteBlock) a.ew->src[i] = i;
    return;
  }
  const uint32_t nitems = e + total;
  if (nw <= kLdsWords && nitems <= kLdsItems) {
    __shared__ uint32_t lkey[kLdsItems], lslot[kLdsItems];
#pragma unroll
    for (uint32_t u = 0; u < kKeysHeld; ++u) {
      const uint32_t i = u * kEliteBlock + tid;
      if (i < e) lkey[i] = ekey[u];
    }
    for (uint32_t i = kKeysHeld * kEliteBlock + tid; i < e; i += kEliteBlock) lkey[i] = keys[i];
    order_children(a, lst, q, c, en, nw, lbits, hist, lkey, lslot);
    __syncthreads();  // the items are in; the histograms start from zero
    for (uint32_t i = tid; i < 2 * 4096; i += kEliteBlock) hist[i] = 0;
    __syncthreads();
    select_items(a, nitems, kprev, hist, hist + 4096, &s_low,
                 [&](uint32_t i) { return lkey[i]; },
                 [&](uint32_t i) { return i < e ? i : lslot[i]; });
  } else {
    // a large population or a long list: bitmap, prefix counts and items in
    // the scratch area
    uint32_t* gbits = a.scratch;
    uint32_t* gwpre = gbits + nw;
    uint32_t* gkey = gwpre + nw;
    uint32_t* gslot = gkey + a.n;
    for (uint32_t i = tid; i < nw; i += kEliteBlock)
      __hip_atomic_store(&gbits[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (uint32_t u = 0; u < kKeysHeld; ++u) {
      const uint32_t i = u * kEliteBlock + tid;
      if (i < e) gkey[i] = ekey[u];
    }
    for (uint32_t i = kKeysHeld * kEliteBlock + tid; i < e; i += kEliteBlock) gkey[i] = keys[i];
    __syncthreads();  // a clear bitmap
    order_children(a, lst, q, c, en, nw, gbits, gwpre, gkey, gslot);
    __syncthreads();  // the items are in
    select_items(a, nitems, kprev, hist, hist + 4096, &s_low,
                 [&](uint32_t i) { return gkey[i]; },
                 [&](uint32_t i) { return i < e ? i : gslot[i]; });
  }
}

// The arguments of a run's elite selection from its descriptor.
__device__ __host__ __forceinline__ EliteArgs elite_args(const PopDesc& d, uint32_t node) {
  EliteArgs a;
  a.keys_a = d.keys_a;
  a.keys_b = d.keys_b;
  a.st = d.state;
  a.ew = d.ew;
  a.count = d.ecount;
  a.list = d.elist;
  a.scratch = d.escratch;
  a.cap = d.ecap;
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
  elite_select_block(elite_args(d, node));
}

hipError_t launch_elite_select(const PopDesc& d, uint32_t node, hipStream_t s) {
  hipLaunchKernelGGL(elite_select_kernel, dim3(1), dim3(kEliteBlock), 0, s, elite_args(d, node));
  return hipGetLastError();
}

hipError_t launch_elite_select_multi(const PopDesc* descs_dev, const uint32_t* runs,
                                     uint32_t count, uint32_t node, hipStream_t s) {
  hipLaunchKernelGGL(elite_select_multi_kernel, dim3(count), dim3(kEliteBlock), 0, s, descs_dev,
                     runs, node);
  return hipGetLastError();
}

}  // namespace ga
