// ga_children.h -- one generation's children: parent selection,
// column-exchange crossover (Sec. 3.4), pair-flip mutation (Sec. 3.5) and
// the child's fitness (Sec. 3.2), fused in one kernel with L lanes per child
// (2, 4 or 8 for orders up to 32; 4 or 8 for orders 36..64; 8 or 16 for
// orders 68..128).  Templates only: the ga_children_*.hip files instantiate
// them for their orders.
// Launch `node` of a chunk produces generation G = gen_base + node + 1 from
// generation G - 1; a wave that makes a child of fitness 0 lowers the run's
// found_gen to G.
#pragma once

#include <hip/hip_runtime.h>

#include "ga_common.h"
#include "ga_device.h"

namespace ga {

// ---------------------------------------------------------------------------
// L lanes per child, 2L per child pair; one word per column up to order 32,
// two up to 64, four (one 16-byte group) above.
//
// Lane 2Lg + t of a block works on pair g of the block: child c = t / L,
// part l = t for child 0 and 2L-1 - t for child 1, so the lanes holding part
// l of the two siblings are mirror images within the 2L lanes (one DPP
// mirror).  Part v of an individual is its 16-byte word group v; lane part l
// holds groups l, l+L, ...  Each quad of lanes computes the pair's four
// Philox blocks, one per lane (quad position 0: selection, 1: crossover, 2
// and 3: mutation of child 0 and 1), and shares them by DPP broadcasts.  A
// tournament reads the contestants' keys first and then only the winner's
// columns.  For the fitness the child is staged in LDS, and lane l takes the
// column pairs (i, i + d mod C), C = M - 1 odd, d = 1 .. (C-1)/2, for i in
// its L-th of 0 .. C-1: every unordered pair of columns 1 .. M-1 exactly
// once.  The child's lanes then add their partial sums.  Above order 64 a
// lane holds its first columns and a sliding window of the partners, one
// new column per distance (lane_pair_sums_w4).
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

// Quad position S's value in all four lanes of each quad.
template <int S>
__device__ __forceinline__ U4 quad_bcast(const U4& v) {
  constexpr int C = S | (S << 2) | (S << 4) | (S << 6);
  return U4{dpp_mov<C>(v.x), dpp_mov<C>(v.y), dpp_mov<C>(v.z), dpp_mov<C>(v.w)};
}

// The value of lane 31 - t of each 32 lanes (bitmask swizzle: and 0x1F,
// or 0, xor 0x1F).
__device__ __forceinline__ uint32_t mirror32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (0x1F << 10));
}

template <int M, int L_>
struct Lanes {
  static constexpr int W = (int)col_words(M);  // words per column
  static constexpr int WL = (M + 31) / 32;     // of them holding rows
  static constexpr int L = L_;                 // lanes per child
  static_assert(W == 1   ? (L == 2 || L == 4 || L == 8)
                : W == 2 ? (L == 4 || L == 8)
                         : (L == 8 || L == 16),
                "lanes per child");
  static constexpr int CPB = 64 / L;           // children per block (one wave)
  static constexpr int P4 = M * W / 4;         // 16-byte groups per individual
  static constexpr int NP = (P4 + L - 1) / L;  // groups per lane
  static constexpr int F = 4 * NP;             // words per lane
  static constexpr int C = M - 1;              // columns 1 .. M-1
  static constexpr int D = (C - 1) / 2;        // pair distances
  static constexpr int K = (C + L - 1) / L;    // first columns per lane
  static __device__ __forceinline__ bool has(int s, uint32_t l) {
    return (s + 1) * L <= P4 || l + (uint32_t)(L * s) < (uint32_t)P4;
  }
  // the sibling lane's value (lane 2L-1 - t of the 2L lanes): quad
  // permutation [3,2,1,0], half-row mirror, row mirror or 32-lane mirror
  static __device__ __forceinline__ uint32_t mirror(uint32_t v) {
    if (L == 2) return dpp_mov<0x1B>(v);
    if (L == 4) return dpp_mov<0x141>(v);
    if (L == 8) return dpp_mov<0x140>(v);
    return mirror32(v);
  }
  // sum over the child's L lanes, in every one of them
  static __device__ __forceinline__ uint32_t sum(uint32_t v) {
    v += dpp_mov<0xB1>(v);                // lane ^ 1
    if (L >= 4) v += dpp_mov<0x4E>(v);    // lane ^ 2
    if (L >= 8) v += dpp_mov<0x141>(v);   // the other quad of the eight
    if (L == 16) v += dpp_mov<0x140>(v);  // the other eight of the row
    return v;
  }
};

// Stores of a child's row and key: nontemporal when NT.  A single run's next
// launch reads them at random slots, mostly from other XCDs; with the mark
// their lines do not linger dirty in the writer's L2, and a tournament
// generation at m = 20, n = 40,000 takes 10% less time (17% at m = 36).
// The batched launch measured 7% slower with the mark, so it stores plainly.
// (The choice is made at compile time: a run-time choice between the two
// stores is merged into one plain store by the compiler.)
template <bool NT>
__device__ __forceinline__ void store_row(uint4* p, const uint4& v) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  if constexpr (NT)
    __builtin_nontemporal_store(v4u{v.x, v.y, v.z, v.w}, reinterpret_cast<v4u*>(p));
  else
    *p = v;
}
template <bool NT>
__device__ __forceinline__ void store_key(uint32_t* p, uint32_t v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Winner of tournament c of pair p (t contestants, draws c*t .. c*t+t-1 of
// the pair's selection stream; block 0 is given): smallest key, then
// smallest index.
__device__ __forceinline__ uint32_t tournament(const PopDesc& d, uint32_t G,
                                               uint32_t p, uint32_t c,
                                               const U4& sel,
                                               const uint32_t* kin) {
  if (d.t == 2) {
    const uint32_t x0 = bounded(c ? sel.z : sel.x, d.n);
    const uint32_t x1 = bounded(c ? sel.w : sel.y, d.n);
    const uint32_t k0 = kin[x0], k1 = kin[x1];
    return (k1 < k0 || (k1 == k0 && x1 < x0)) ? x1 : x0;
  }
  DrawSeq ds(d.seed, kStreamSelect, G, p, sel);
  uint32_t bx = bounded(ds.at(c * d.t), d.n);
  uint32_t bk = kin[bx];
  for (uint32_t k = 1; k < d.t; ++k) {
    const uint32_t x = bounded(ds.at(c * d.t + k), d.n);
    const uint32_t kx = kin[x];
    if (kx < bk || (kx == bk && x < bx)) {
      bx = x;
      bk = kx;
    }
  }
  return bx;
}

// The words a lane holds of a child of order M with L lanes per child.
template <int M, int L_>
using LaneWords = uint32_t[Lanes<M, L_>::F];

// Pair-flip mutation (Sec. 3.5, third method) of a child held as parts: the
// lane holding the chosen column flips it; the draws are those of the
// one-lane form (columns at draws 0 .. nc-1, row pairs after them).  One
// row pair (r1, r2) on column `col` given the flips `mask` chosen so far;
// `apply` writes the column back.

template <int M, int L_>
__device__ __forceinline__ void flip_parts(LaneWords<M, L_>& f,
                                           uint32_t l, uint32_t col,
                                           uint32_t r1, uint32_t r2,
                                           uint64_t& mask, bool apply) {
  using Q = Lanes<M, L_>;
  constexpr int F = Q::F, W = Q::W, L = Q::L;
  const uint32_t w0 = col * W;                       // first word in the row
  const uint32_t v = w0 >> 2;                        // its 16-byte group
  const uint32_t k = (v / L) * 4 + (w0 & 3u);        // word in this lane
  uint64_t x = 0;
  [&]<int... J>(std::integer_sequence<int, J...>) __attribute__((always_inline)) {
    uint32_t lo = 0, hi = 0;
    ((lo |= pick_if_eq<J>(k, f[J])), ...);
    if (W == 2) ((hi |= pick_if_eq<J>(k + 1, f[J])), ...);
    x = (uint64_t)lo | ((uint64_t)hi << 32);
  }(std::make_integer_sequence<int, F>{});
  const uint64_t y = x ^ mask;
  if (((y >> r1) ^ (y >> r2)) & 1u) mask ^= (1ull << r1) | (1ull << r2);
  if (!apply) return;
  const uint64_t mk = (v % L) == l ? mask : 0ull;  // another lane holds it
  [&]<int... J>(std::integer_sequence<int, J...>) __attribute__((always_inline)) {
    ((f[J] ^= pick_if_eq<J>(k, (uint32_t)mk)), ...);
    if (W == 2) ((f[J] ^= pick_if_eq<J>(k + 1, (uint32_t)(mk >> 32))), ...);
  }(std::make_integer_sequence<int, F>{});
}

// The same for four-word columns (orders above 64): the column is the
// lane's group col / L, the flips so far a 128-bit mask of four words.
template <int M, int L_>
__device__ __forceinline__ void flip_parts4(LaneWords<M, L_>& f,
                                            uint32_t l, uint32_t col,
                                            uint32_t r1, uint32_t r2,
                                            uint32_t (&mask)[4], bool apply) {
  using Q = Lanes<M, L_>;
  constexpr int NP = Q::NP, L = Q::L;
  const uint32_t grp = col / L;  // the column's group in the lane holding it
  uint32_t x[4] = {0, 0, 0, 0};
  [&]<int... S>(std::integer_sequence<int, S...>) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) ((x[e] |= pick_if_eq<S>(grp, f[4 * S + e])), ...);
  }(std::make_integer_sequence<int, NP>{});
  const U4 y{x[0] ^ mask[0], x[1] ^ mask[1], x[2] ^ mask[2], x[3] ^ mask[3]};
  const uint32_t b1 = (y[r1 >> 5] >> (r1 & 31u)) & 1u;
  const uint32_t b2 = (y[r2 >> 5] >> (r2 & 31u)) & 1u;
  if (b1 != b2) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      mask[e] ^= ((r1 >> 5) == (uint32_t)e ? 1u << (r1 & 31u) : 0u) ^
                 ((r2 >> 5) == (uint32_t)e ? 1u << (r2 & 31u) : 0u);
  }
  if (!apply || col % L != l) return;  // another lane holds the column
  [&]<int... S>(std::integer_sequence<int, S...>) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < 4; ++e) ((f[4 * S + e] ^= pick_if_eq<S>(grp, mask[e])), ...);
  }(std::make_integer_sequence<int, NP>{});
}

template <int M, int L_>
__device__ __forceinline__ void mutate_parts4(LaneWords<M, L_>& f,
                                              uint32_t l, DrawSeq& ds,
                                              uint32_t nc, uint32_t nr) {
  if (nc == 1 && nr == 1) {  // draws 0, 1, 2: all in the given block 0
    uint32_t mask[4] = {0, 0, 0, 0};
    flip_parts4<M, L_>(f, l, 1u + bounded(ds.cur.x, M - 1), bounded(ds.cur.y, M),
                       bounded(ds.cur.z, M), mask, true);
    return;
  }
  for (uint32_t jc = 0; jc < nc; ++jc) {
    const uint32_t col = 1u + bounded(ds.at(jc), M - 1);
    uint32_t mask[4] = {0, 0, 0, 0};
    for (uint32_t ir = 0; ir < nr; ++ir)
      flip_parts4<M, L_>(f, l, col, bounded(ds.at(nc + 2 * ir), M),
                         bounded(ds.at(nc + 2 * ir + 1), M), mask, ir + 1 == nr);
  }
}

template <int M, int L_>
__device__ __forceinline__ void mutate_parts(LaneWords<M, L_>& f,
                                             uint32_t l, DrawSeq& ds,
                                             uint32_t nc, uint32_t nr) {
  if constexpr (Lanes<M, L_>::W == 4) {
    mutate_parts4<M, L_>(f, l, ds, nc, nr);
  } else {
    if (nc == 1 && nr == 1) {  // draws 0, 1, 2: all in the given block 0
      uint64_t mask = 0;
      flip_parts<M, L_>(f, l, 1u + bounded(ds.cur.x, M - 1), bounded(ds.cur.y, M),
                        bounded(ds.cur.z, M), mask, true);
      return;
    }
    for (uint32_t jc = 0; jc < nc; ++jc) {
      const uint32_t col = 1u + bounded(ds.at(jc), M - 1);
      uint64_t mask = 0;
      for (uint32_t ir = 0; ir < nr; ++ir)
        flip_parts<M, L_>(f, l, col, bounded(ds.at(nc + 2 * ir), M),
                          bounded(ds.at(nc + 2 * ir + 1), M), mask, ir + 1 == nr);
    }
  }
}

// This lane's share of the column-pair sums of the child staged at `me`.
template <int M, uint32_t NEED, int L_>
__device__ __forceinline__ Sums lane_pair_sums(const uint32_t* me, uint32_t l) {
  using Q = Lanes<M, L_>;
  constexpr int C = Q::C, D = Q::D, K = Q::K, L = Q::L, W = Q::W, H = M / 2;
  const uint32_t r = l * K;
  uint32_t z[K + D][W];
#pragma unroll
  for (int k = 0; k < K + D; ++k) {
    const uint32_t i = (r + k) % (uint32_t)C;
    if (W == 1) {
      z[k][0] = me[1 + i];
    } else {
      const uint2 v = reinterpret_cast<const uint2*>(me)[1 + i];
      z[k][0] = v.x;
      z[k][W - 1] = v.y;
    }
  }
  Sums s{0, 0, 0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (k + (L - 1) * K < C) {  // column r + k exists in every lane
#pragma unroll
      for (int dd = 1; dd <= D; ++dd)
        pair_step<NEED>(z[k][0] ^ z[k + dd][0], z[k][W - 1] ^ z[k + dd][W - 1], W, H, s);
    } else {
      Sums g{0, 0, 0};
#pragma unroll
      for (int dd = 1; dd <= D; ++dd)
        pair_step<NEED>(z[k][0] ^ z[k + dd][0], z[k][W - 1] ^ z[k + dd][W - 1], W, H, g);
      const bool in = r + k < (uint32_t)C;
      s.sq += in ? g.sq : 0u;
      s.ab += in ? g.ab : 0u;
      s.nz += in ? g.nz : 0u;
    }
  }
  return s;
}

// The same for four-word columns (orders above 64).  Lane l owns columns
// r + k (k < K, r = l K; past C - 1 a zero column, which adds d = 0 against
// any balanced partner), and a ring of K partner columns: before distance
// dd it holds columns r + dd .. r + dd + K - 1, slot t % K for column r + t,
// so each distance loads one column and every operand index is fixed at
// compile time.  The distances run in blocks of K, then a tail of D % K.
template <int M, uint32_t NEED, int L_>
__device__ __forceinline__ Sums lane_pair_sums_w4(const uint32_t* me, uint32_t l) {
  using Q = Lanes<M, L_>;
  constexpr int C = Q::C, D = Q::D, K = Q::K, WL = Q::WL, H = M / 2;
  const uint4* col = reinterpret_cast<const uint4*>(me) + 1;  // columns 1 .. C
  const uint32_t r = l * K;
  uint4 a[K], b[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t i = r + k;
    b[k] = col[i % C];
    a[k] = i < (uint32_t)C ? b[k] : make_uint4(0, 0, 0, 0);
  }
  uint32_t nxt = (r + K) % C;  // column of ring entry t = dd + K - 1
  Sums s{0, 0, 0};
  constexpr int NB = D / K, TAIL = D % K;
#pragma unroll 1
  for (int blk = 0; blk < NB; ++blk) {
#pragma unroll
    for (int j = 0; j < K; ++j) {  // distance dd = blk K + j + 1
      b[j] = col[nxt];
      nxt = nxt + 1 == (uint32_t)C ? 0u : nxt + 1;
#pragma unroll
      for (int k = 0; k < K; ++k) pair_step4<NEED, WL>(a[k], b[(k + j + 1) % K], H, s);
    }
  }
#pragma unroll
  for (int j = 0; j < TAIL; ++j) {
    b[j] = col[nxt];
    nxt = nxt + 1 == (uint32_t)C ? 0u : nxt + 1;
#pragma unroll
    for (int k = 0; k < K; ++k) pair_step4<NEED, WL>(a[k], b[(k + j + 1) % K], H, s);
  }
  return s;
}

template <int M, uint32_t NEED, int L_>
__device__ __forceinline__ uint32_t lanes_fitness_need(const uint32_t* me,
                                                       uint32_t l, uint32_t kind) {
  using Q = Lanes<M, L_>;
  Sums s;
  if constexpr (Q::W == 4)
    s = lane_pair_sums_w4<M, NEED, L_>(me, l);
  else
    s = lane_pair_sums<M, NEED, L_>(me, l);
  if (NEED & kNeedSQ) s.sq = Q::sum(s.sq);
  if (NEED & kNeedABS) s.ab = Q::sum(s.ab);
  if (NEED & kNeedNNZ) s.nz = Q::sum(s.nz);
  return key_of(kind, s);
}

// Key of the staged child.  NEED = 0: the sums are chosen at run time.
template <int M, uint32_t NEED, int L_>
__device__ __forceinline__ uint32_t lanes_fitness(const uint32_t* me, uint32_t l,
                                                  uint32_t kind) {
  if (NEED) return lanes_fitness_need<M, NEED, L_>(me, l, kind);
  switch (needs_of_kind(kind)) {  // uniform over the launch
    case kNeedSQ: return lanes_fitness_need<M, kNeedSQ, L_>(me, l, kind);
    case kNeedABS: return lanes_fitness_need<M, kNeedABS, L_>(me, l, kind);
    case kNeedNNZ: return lanes_fitness_need<M, kNeedNNZ, L_>(me, l, kind);
    default: return lanes_fitness_need<M, kNeedSQ | kNeedNNZ, L_>(me, l, kind);
  }
}

// The child of this lane's group in generation G; `lds` holds the block's
// children (M*W words each).  Lanes of pairs past the last compute a copy of
// the last pair and store nothing.  NT: nontemporal stores of the child.
template <int M, uint32_t NEED, int L_, bool NT>
__device__ __forceinline__ unsigned long long child(const PopDesc& d, uint32_t G,
                                                   uint32_t node, uint32_t* lds) {
  using Q = Lanes<M, L_>;
  constexpr int L = Q::L, NP = Q::NP;
  constexpr uint32_t MW = M * Q::W;
  const bool odd_in = ((G - 1) & 1u) != 0;
  const uint32_t* pin = odd_in ? d.pop_b : d.pop_a;
  const uint32_t* kin = odd_in ? d.keys_b : d.keys_a;
  uint32_t* pout = odd_in ? d.pop_a : d.pop_b;
  uint32_t* kout = odd_in ? d.keys_a : d.keys_b;
  const uint32_t lane = threadIdx.x, t = lane & (2 * L - 1), u = lane & 3u;
  const uint32_t c = t / L, l = c ? 2 * L - 1 - t : t;
  const uint32_t g = lane / (2 * L);
  const uint32_t pw = (blockIdx.x - d.block_begin) * (Q::CPB / 2) + g;
  const uint32_t npairs = (d.nchild + 1) >> 1;
  const uint32_t p = min(pw, npairs - 1);
  const uint32_t q = 2 * p + c;
  const bool valid = 2 * pw + c < d.nchild;

  const uint32_t stream = u == 0 ? kStreamSelect : (u == 1 ? kStreamXover : kStreamMutate);
  const uint32_t mq = d.mut_shared ? kSharedMutation : 2 * p + (u - 2);
  const U4 blk = draw_block(d.seed, stream, G, u < 2 ? p : mq, 0);
  const U4 sel = quad_bcast<0>(blk);
  const U4 xo = quad_bcast<1>(blk);
  const U4 mb0 = quad_bcast<2>(blk), mb1 = quad_bcast<3>(blk);

  // this child's first parent (its columns before the cut) and slot
  const uint32_t* first;
  uint32_t dst;
  uint32_t pslot = ~0u, pkey = 0;  // with d.psel: the parent slot this lane group fills
  if (d.paper) {
    const uint32_t N = d.n / 4;
    const uint32_t ps = c ? p + N : p;
    if (d.psel) {  // parent slot ps receives sel[pi(ps)] of generation G - 1
      const uint32_t src = d.psel[d.pfwd[(size_t)node * (2 * N) + ps]];
      first = pin + (size_t)src * MW;
      pkey = kin[src];
      pslot = ps;
    } else {
      first = pout + (size_t)ps * MW;
    }
    dst = (c ? 3u * N : 2u * N) + p;
  } else {
    first = pin + (size_t)tournament(d, G, p, c, sel, kin) * MW;
    dst = d.elite + q;
  }
  const uint4* f4 = reinterpret_cast<const uint4*>(first);
  uint32_t f[Q::F];
#pragma unroll
  for (int s = 0; s < NP; ++s) {
    uint4 v = make_uint4(0, 0, 0, 0);
    if (Q::has(s, l)) v = f4[l + L * s];
    f[4 * s] = v.x;
    f[4 * s + 1] = v.y;
    f[4 * s + 2] = v.z;
    f[4 * s + 3] = v.w;
  }
  if (pslot != ~0u && valid) {  // the parent itself, into its slot of generation G
    uint4* p4 = reinterpret_cast<uint4*>(pout + (size_t)pslot * MW);
#pragma unroll
    for (int s = 0; s < NP; ++s)
      if (Q::has(s, l))
        store_row<NT>(p4 + l + L * s, make_uint4(f[4 * s], f[4 * s + 1], f[4 * s + 2], f[4 * s + 3]));
    if (l == 0) store_key<NT>(kout + pslot, pkey);
  }
  // column-exchange crossover (Sec. 3.4): columns >= cut from the sibling's
  // first parent
  const uint32_t cut =
      ((uint64_t)xo.x < d.xo_thr) ? 1u + bounded(xo.y, M - 1) : (uint32_t)M;
#pragma unroll
  for (int s = 0; s < NP; ++s) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t o = Q::mirror(f[4 * s + e]);
      const uint32_t col = (4u * (l + L * s) + e) / Q::W;
      f[4 * s + e] = col < cut ? f[4 * s + e] : o;
    }
  }
  if ((uint64_t)(c ? xo.w : xo.z) < d.mut_thr) {
    DrawSeq ds(d.seed, kStreamMutate, G, d.mut_shared ? kSharedMutation : q, c ? mb1 : mb0);
    mutate_parts<M, L_>(f, l, ds, d.nc, d.nr);
  }
  uint32_t* me = lds + (g * 2 + c) * MW;
  uint4* o4 = reinterpret_cast<uint4*>(pout + (size_t)dst * MW);
  if constexpr (Q::W == 4) {  // store now: the words are dead in the fitness
    if (valid) {
#pragma unroll
      for (int s = 0; s < NP; ++s)
        if (Q::has(s, l))
          store_row<NT>(o4 + l + L * s,
                    make_uint4(f[4 * s], f[4 * s + 1], f[4 * s + 2], f[4 * s + 3]));
    }
  }
#pragma unroll
  for (int s = 0; s < NP; ++s)
    if (Q::has(s, l))
      reinterpret_cast<uint4*>(me)[l + L * s] =
          make_uint4(f[4 * s], f[4 * s + 1], f[4 * s + 2], f[4 * s + 3]);
  __syncthreads();
  const uint32_t key = lanes_fitness<M, NEED, L_>(me, l, d.kind);
  if (!valid) return ~0ull;
  if constexpr (Q::W != 4) {
#pragma unroll
    for (int s = 0; s < NP; ++s)
      if (Q::has(s, l))
        store_row<NT>(o4 + l + L * s,
                  make_uint4(f[4 * s], f[4 * s + 1], f[4 * s + 2], f[4 * s + 3]));
  }
  if (l == 0) store_key<NT>(kout + dst, key);
  // elitism in ga_run: a child below the largest elite key may be among the
  // next elites; the block's such children go to its candidate list, with
  // one atomic for all of them
  if (d.ecount) {
    const bool cand = l == 0 && key < d.ew->kstar;
    const unsigned long long bal = __ballot(cand);
    if (bal) {
      const uint32_t list = (blockIdx.x - d.block_begin) % kEliteLists;
      const int leader = __ffsll((long long)bal) - 1;
      uint32_t base = 0;
      if ((int)lane == leader) base = atomicAdd(&d.ecount[list], (uint32_t)__popcll(bal));
      base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
      if (cand) {
        const uint32_t rank = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        d.elist[(size_t)list * d.ecap + base + rank] = make_uint2(dst, key);
      }
    }
  }
  return ((unsigned long long)key << 32) | dst;
}

// Elitism in ga_run: block b copies elites b, b + nblocks, ... of generation
// G (rows ew->src[s] of G - 1, with their keys) into slots s.  The block's
// first elite is loaded before its child is made (load_first_elite) and
// stored after (copy_elites), so the copy adds no round trip of its own.
struct EliteRow {
  uint4 v;       // this lane's 16-byte group of the row (lanes < V)
  uint32_t key;  // its key (lane 0)
};
template <int M>
__device__ __forceinline__ EliteRow load_first_elite(const PopDesc& d, uint32_t G) {
  constexpr uint32_t V = M * col_words(M) / 4;  // 16-byte groups per row
  EliteRow r{make_uint4(0, 0, 0, 0), 0u};
  const uint32_t s = blockIdx.x - d.block_begin;
  if (s >= d.elite) return r;
  const bool odd_in = ((G - 1) & 1u) != 0;
  const uint4* pin = reinterpret_cast<const uint4*>(odd_in ? d.pop_b : d.pop_a);
  const uint32_t* kin = odd_in ? d.keys_b : d.keys_a;
  const uint32_t src = d.ew->src[s];
  if (threadIdx.x < V) r.v = pin[(size_t)src * V + threadIdx.x];
  if (threadIdx.x == 0) r.key = kin[src];
  return r;
}
template <int M, bool NT>
__device__ __forceinline__ void copy_elites(const PopDesc& d, uint32_t G, const EliteRow& first) {
  constexpr uint32_t V = M * col_words(M) / 4;
  const bool odd_in = ((G - 1) & 1u) != 0;
  const uint4* pin = reinterpret_cast<const uint4*>(odd_in ? d.pop_b : d.pop_a);
  const uint32_t* kin = odd_in ? d.keys_b : d.keys_a;
  uint4* pout = reinterpret_cast<uint4*>(odd_in ? d.pop_a : d.pop_b);
  uint32_t* kout = odd_in ? d.keys_a : d.keys_b;
  uint32_t s = blockIdx.x - d.block_begin;
  if (s >= d.elite) return;
  if (threadIdx.x < V) store_row<NT>(pout + (size_t)s * V + threadIdx.x, first.v);
  if (threadIdx.x == 0) store_key<NT>(kout + s, first.key);
  for (uint32_t v = kChildBlock + threadIdx.x; v < V; v += kChildBlock) {
    const uint32_t src = d.ew->src[s];
    store_row<NT>(pout + (size_t)s * V + v, pin[(size_t)src * V + v]);
  }
  for (s += d.nblocks; s < d.elite; s += d.nblocks) {
    const uint32_t src = d.ew->src[s];
    for (uint32_t v = threadIdx.x; v < V; v += kChildBlock)
      store_row<NT>(pout + (size_t)s * V + v, pin[(size_t)src * V + v]);
    if (threadIdx.x == 0) store_key<NT>(kout + s, kin[src]);
  }
}

// Generation G of launch `node`, and whether it runs (see RunState).  The
// state was last written by an earlier kernel, so plain loads see it.
__device__ __forceinline__ bool generation_of(const PopDesc& d, uint32_t node,
                                              uint32_t* G) {
  const uint2 v = *reinterpret_cast<const uint2*>(&d.state->gen_base);
  *G = v.x + node + 1;  // v.x = gen_base, v.y = found_gen
  if (*G > d.max_gen) return false;
  if (d.stop_on_found && v.y < *G) return false;
  return true;
}

// The block's children (one wave); a wave holding a key of 0 records it.
template <typename F>
__device__ __forceinline__ void children_block(const PopDesc& d, uint32_t node,
                                               F&& body) {
  uint32_t G;
  if (!generation_of(d, node, &G)) return;  // uniform over the launch
  const unsigned long long b = body(G);
  if (d.stop_on_found) note_zero(d.state, b, G);
}

// One population of order M, L lanes per child, the sums its fitness kind
// needs fixed at compile time, descriptor by value.
template <int M, uint32_t NEED, int L>
__global__ __launch_bounds__(kChildBlock) void children_one_kernel(PopDesc d,
                                                                   uint32_t node) {
  using Q = Lanes<M, L>;
  __shared__ __align__(16) uint32_t lds[Q::CPB * M * Q::W];
  children_block(d, node, [&](uint32_t G) __attribute__((always_inline)) {
    EliteRow er{make_uint4(0, 0, 0, 0), 0u};
    if (d.ew) er = load_first_elite<M>(d, G);
    const unsigned long long b = child<M, NEED, L, true>(d, G, node, lds);
    if (d.ew) copy_elites<M, true>(d, G, er);
    return b;
  });
}

// Several populations of order M, L lanes per child, in one launch (block ->
// population through block_pop).  One instantiation per order keeps every kernel free of calls:
// with all orders behind one switch the compiler outlines the body into a
// function longer than the reach of a conditional branch, and the long
// branches it then emits reuse the return-address registers, so the
// function never returns.
template <int M, int L>
__global__ __launch_bounds__(kChildBlock) void children_multi_kernel(
    const PopDesc* __restrict__ descs, const uint32_t* __restrict__ block_pop,
    uint32_t node) {
  using Q = Lanes<M, L>;
  __shared__ __align__(16) uint32_t lds[Q::CPB * M * Q::W];
  const PopDesc d = descs[block_pop[blockIdx.x]];
  children_block(d, node, [&](uint32_t G) __attribute__((always_inline)) {
    const unsigned long long b = child<M, 0, L, false>(d, G, node, lds);
    // the elites after the child: a row held across it would cost this
    // kernel's occupancy (it keeps the fitness kind as a run-time choice)
    if (d.ew) copy_elites<M, false>(d, G, load_first_elite<M>(d, G));
    return b;
  });
}

template <int M, int L>
hipError_t launch_one_lanes(const PopDesc& d, uint32_t node, hipStream_t s) {
  const dim3 grid(d.nblocks), block(kChildBlock);
  if constexpr (M > 64) {  // one kernel per tile shape; the kind is chosen inside
    hipLaunchKernelGGL((children_one_kernel<M, 0u, L>), grid, block, 0, s, d, node);
  } else {
    switch (needs_of_kind(d.kind)) {
      case kNeedSQ:
        hipLaunchKernelGGL((children_one_kernel<M, kNeedSQ, L>), grid, block, 0, s, d, node);
        break;
      case kNeedABS:
        hipLaunchKernelGGL((children_one_kernel<M, kNeedABS, L>), grid, block, 0, s, d, node);
        break;
      case kNeedNNZ:
        hipLaunchKernelGGL((children_one_kernel<M, kNeedNNZ, L>), grid, block, 0, s, d, node);
        break;
      default:
        hipLaunchKernelGGL((children_one_kernel<M, kNeedSQ | kNeedNNZ, L>), grid, block, 0,
                           s, d, node);
    }
  }
  return hipGetLastError();
}

// Children of one population of order M (lanes from its descriptor).
template <int M>
hipError_t launch_one_order(const PopDesc& d, uint32_t node, hipStream_t s) {
  switch (d.lanes) {
    case 2:
      if constexpr (M <= 32) return launch_one_lanes<M, 2>(d, node, s);
      return hipErrorInvalidValue;
    case 4:
      if constexpr (M <= 64) return launch_one_lanes<M, 4>(d, node, s);
      return hipErrorInvalidValue;
    case 8: return launch_one_lanes<M, 8>(d, node, s);
    case 16:
      if constexpr (M > 64) return launch_one_lanes<M, 16>(d, node, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// Children of several populations of order M in one launch.
template <int M>
hipError_t launch_multi_order(const PopDesc* descs, const uint32_t* block_pop,
                              uint32_t blocks, uint32_t lanes, uint32_t node,
                              hipStream_t s) {
  const dim3 grid(blocks), block(kChildBlock);
  switch (lanes) {
    case 2:
      if constexpr (M <= 32) {
        hipLaunchKernelGGL((children_multi_kernel<M, 2>), grid, block, 0, s, descs, block_pop,
                           node);
        break;
      }
      return hipErrorInvalidValue;
    case 4:
      if constexpr (M <= 64) {
        hipLaunchKernelGGL((children_multi_kernel<M, 4>), grid, block, 0, s, descs, block_pop,
                           node);
        break;
      }
      return hipErrorInvalidValue;
    case 8:
      hipLaunchKernelGGL((children_multi_kernel<M, 8>), grid, block, 0, s, descs, block_pop, node);
      break;
    case 16:
      if constexpr (M > 64) {
        hipLaunchKernelGGL((children_multi_kernel<M, 16>), grid, block, 0, s, descs, block_pop,
                           node);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Per-order entry points, defined by the ga_children_*.hip files.
#define GA_DECLARE_ORDER(MM)                                                    \
  hipError_t launch_children_one_m##MM(const PopDesc& d, uint32_t node,        \
                                       hipStream_t s);                         \
  hipError_t launch_children_multi_m##MM(const PopDesc* descs,                 \
                                         const uint32_t* block_pop,            \
                                         uint32_t blocks, uint32_t lanes,      \
                                         uint32_t node, hipStream_t s);
#define GA_DEFINE_ORDER(MM)                                                     \
  hipError_t launch_children_one_m##MM(const PopDesc& d, uint32_t node,        \
                                       hipStream_t s) {                        \
    return launch_one_order<MM>(d, node, s);                                    \
  }                                                                             \
  hipError_t launch_children_multi_m##MM(const PopDesc* descs,                 \
                                         const uint32_t* block_pop,            \
                                         uint32_t blocks, uint32_t lanes,      \
                                         uint32_t node, hipStream_t s) {       \
    return launch_multi_order<MM>(descs, block_pop, blocks, lanes, node, s);   \
  }
#define GA_FOR_EACH_ORDER(X)                                                  \
  X(4) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(36) X(40) X(44) X(48) X(52) \
  X(56) X(60) X(64) X(68) X(72) X(76) X(80) X(84) X(88) X(92) X(96) X(100)   \
  X(104) X(108) X(112) X(116) X(120) X(124) X(128)

GA_FOR_EACH_ORDER(GA_DECLARE_ORDER)

}  // namespace ga
