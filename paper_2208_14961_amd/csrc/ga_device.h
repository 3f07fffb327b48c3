// ga_device.h -- device building blocks of libga (gfx950).
//
// Counter-based randomness (Philox4x32-10), bounded draws, and the packed
// Gram + fitness core.  A population is stored packed: column j of a matrix
// of order M is W = col_words(M) uint32 words (1, 2, or 4 above order 64),
// bit r set iff entry (r, j) is -1.  The dot product of columns i and j is M - 2 popcount(x_i ^ x_j)
// (Sec. 3.2 uses the Gram matrix Q^T Q of +-1 columns; this is the same
// number computed on bits).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "ga_internal.h"

namespace ga {

// Philox stream tags (the "stream" word of the counter).
enum : uint32_t {
  kStreamInit = 1,
  kStreamSelect = 2,
  kStreamXover = 3,
  kStreamMutate = 4,
  kStreamPerm = 5
};

// Draw index of the mutation shared by a whole generation (GA_MUT_SHARED),
// above every child index.
constexpr uint32_t kSharedMutation = 0xFFFFFFFFu;

// Fitness kinds (same numbering as the public header).
enum : uint32_t {
  kFitSQ = 0,
  kFitABS = 1,
  kFitNNZ = 2,
  kFitSQNNZ = 3,
  kFitF1 = 4,
  kFitF2 = 5
};

// Which running sums a kind needs.
enum : uint32_t { kNeedSQ = 1, kNeedABS = 2, kNeedNNZ = 4 };

__host__ __device__ inline uint32_t needs_of_kind(uint32_t kind) {
  switch (kind) {
    case kFitSQ: return kNeedSQ;
    case kFitABS: return kNeedABS;
    case kFitNNZ: return kNeedNNZ;
    case kFitSQNNZ: return kNeedSQ | kNeedNNZ;
    case kFitF1: return kNeedABS;
    default: return kNeedNNZ;  // kFitF2
  }
}

struct U4 {
  uint32_t x, y, z, w;
  // Word i (0..3) by selects: written as plain conditionals the compiler
  // may copy the four words to scratch and index them there.
  __device__ uint32_t operator[](uint32_t i) const {
    uint32_t r;
    asm("v_cmp_eq_u32 vcc, 1, %1\n\t"
        "v_cndmask_b32 %0, %2, %3, vcc\n\t"
        "v_cmp_eq_u32 vcc, 2, %1\n\t"
        "v_cndmask_b32 %0, %0, %4, vcc\n\t"
        "v_cmp_eq_u32 vcc, 3, %1\n\t"
        "v_cndmask_b32 %0, %0, %5, vcc"
        : "=&v"(r)
        : "v"(i), "v"(x), "v"(y), "v"(z), "v"(w)
        : "vcc");
    return r;
  }
};

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products of counter words 0 and 2, the high halves xor'ed with words 1, 3
// and the round key into the new words 0, 2, the low halves becoming words
// 1, 3; the key advances by the Weyl constants 0x9E3779B9, 0xBB67AE85.
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2,
                                     uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// Block `blk` (= draw index / 4) of (stream, generation, index).
__device__ __forceinline__ U4 draw_block(uint64_t seed, uint32_t stream,
                                         uint32_t gen, uint32_t idx,
                                         uint32_t blk) {
  return philox(blk, idx, gen, stream, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// floor(u * range / 2^32): an integer in [0, range).
__device__ __forceinline__ uint32_t bounded(uint32_t u, uint32_t range) {
  return __umulhi(u, range);
}

// Sequential reader of draws d = 0, 1, 2, ... of one (stream, gen, index),
// computing each Philox block once.
struct DrawSeq {
  uint64_t seed;
  uint32_t stream, gen, idx;
  uint32_t blk;
  U4 cur;
  __device__ DrawSeq(uint64_t s, uint32_t st, uint32_t g, uint32_t i)
      : seed(s), stream(st), gen(g), idx(i), blk(0xffffffffu) {}
  // starts with block 0 already computed
  __device__ DrawSeq(uint64_t s, uint32_t st, uint32_t g, uint32_t i, U4 b0)
      : seed(s), stream(st), gen(g), idx(i), blk(0), cur(b0) {}
  __device__ uint32_t at(uint32_t d) {
    const uint32_t b = d >> 2;
    if (b != blk) {
      cur = draw_block(seed, stream, gen, idx, b);
      blk = b;
    }
    return cur[d & 3u];
  }
};

// ---------------------------------------------------------------------------
// Packed Gram + fitness.  Columns 1..M-1 only: under the invariants column 0
// is all +1 and every other column balanced, so c_0 . c_j = 0.
// For a pair (i, j) with p = popcount(x_i ^ x_j) the dot product is
// g = M - 2p = -2 d with d = p - M/2, hence g^2 = 4 d^2, |g| = 2 |d|,
// g != 0 iff d != 0.
// ---------------------------------------------------------------------------
template <int M>
struct Cols {
  static constexpr int W = (int)col_words(M);
  uint32_t w[M][W];
};

struct Sums {
  uint32_t sq;   // sum of d^2
  uint32_t ab;   // sum of |d|
  uint32_t nz;   // number of d != 0
};

// One accumulation step per pair.  Written as single instructions so the
// sums stay sequential chains: left to the compiler, a sum of hundreds of
// terms is reassociated into a tree that keeps every term live at once.
// d = popcount - H is produced by v_bcnt_u32_b32's add operand.
__device__ __forceinline__ uint32_t acc_sq(uint32_t acc, int d) {
  asm("v_mad_i32_i24 %0, %1, %1, %0" : "+v"(acc) : "v"(d));
  return acc;
}
__device__ __forceinline__ uint32_t acc_abs(uint32_t acc, uint32_t pc,
                                            uint32_t h) {
  asm("v_sad_u32 %0, %1, %2, %0" : "+v"(acc) : "v"(pc), "s"(h));
  return acc;
}
__device__ __forceinline__ uint32_t acc_nz(uint32_t acc, int d) {
  asm("v_cmp_ne_u32 vcc, 0, %1\n\tv_addc_co_u32 %0, vcc, 0, %0, vcc"
      : "+v"(acc)
      : "v"(d)
      : "vcc");
  return acc;
}

// Contribution of one column pair given the xor of its words (p = popcount).
template <uint32_t NEED>
__device__ __forceinline__ void pair_step(uint32_t x0, uint32_t x1, int W,
                                          int H, Sums& s) {
  if (NEED == kNeedABS) {
    const uint32_t p = W > 1 ? __popc(x0) + __popc(x1) : __popc(x0);
    s.ab = acc_abs(s.ab, p, (uint32_t)H);
    return;
  }
  const int d = (W > 1 ? (int)__popc(x0) + (int)__popc(x1) : (int)__popc(x0)) - H;
  if (NEED & kNeedSQ) s.sq = acc_sq(s.sq, d);
  if (NEED & kNeedABS) s.ab = acc_abs(s.ab, (uint32_t)(d + H), (uint32_t)H);
  if (NEED & kNeedNNZ) s.nz = acc_nz(s.nz, d);
}

// The same for columns of four words (orders above 64); the first WL words
// hold rows, the rest are 0.
template <uint32_t NEED, int WL>
__device__ __forceinline__ void pair_step4(const uint4& a, const uint4& b, int H,
                                           Sums& s) {
  // One chain of v_bcnt_u32_b32 accumulates, starting from -H for the kinds
  // that use d = p - H.  Left to itself the compiler takes each popcount
  // with a zero addend and sums them with three-input adds: 10 issue slots
  // where the chain takes 8.
  uint32_t p = NEED == kNeedABS ? 0u : (uint32_t)(-H);
  asm("v_bcnt_u32_b32 %0, %1, %0" : "+v"(p) : "v"(a.x ^ b.x));
  asm("v_bcnt_u32_b32 %0, %1, %0" : "+v"(p) : "v"(a.y ^ b.y));
  asm("v_bcnt_u32_b32 %0, %1, %0" : "+v"(p) : "v"(a.z ^ b.z));
  if (WL == 4) asm("v_bcnt_u32_b32 %0, %1, %0" : "+v"(p) : "v"(a.w ^ b.w));
  if (NEED == kNeedABS) {
    s.ab = acc_abs(s.ab, p, (uint32_t)H);
    return;
  }
  const int d = (int)p;
  p += (uint32_t)H;
  if (NEED & kNeedSQ) s.sq = acc_sq(s.sq, d);
  if (NEED & kNeedABS) s.ab = acc_abs(s.ab, p, (uint32_t)H);
  if (NEED & kNeedNNZ) s.nz = acc_nz(s.nz, d);
}

// All pairs 1 <= i < j < M of a register-resident individual (M <= 32).
template <int M, uint32_t NEED>
__device__ __forceinline__ Sums pair_sums(const Cols<M>& c) {
  static_assert(M <= 32, "register path holds one word per column");
  Sums s{0, 0, 0};
#pragma unroll
  for (int i = 1; i < M; ++i) {
#pragma unroll
    for (int j = i + 1; j < M; ++j)
      pair_step<NEED>(c.w[i][0] ^ c.w[j][0], 0u, 1, M / 2, s);
  }
  return s;
}

// All pairs of a memory-resident individual of runtime order M (two words
// per column): columns 1..M-1 in blocks of R held in registers, pairs taken
// tile by tile.  Columns past M-1 read as zero words; a zero column against
// a balanced one contributes d = 0, and the C(npad, 2) zero-zero pairs
// contribute d = -H each, which is subtracted at the end.
template <uint32_t NEED, int R>
__device__ __forceinline__ void load_block2(const uint32_t* P, uint32_t M,
                                            uint32_t col0, uint32_t (&x)[R][2]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t col = col0 + r;
    if (col < M) {
      const uint2 v = *reinterpret_cast<const uint2*>(P + 2 * col);
      x[r][0] = v.x;
      x[r][1] = v.y;
    } else {
      x[r][0] = 0;
      x[r][1] = 0;
    }
  }
}

template <uint32_t NEED, int R>
__device__ __forceinline__ Sums blocked_sums_w2(const uint32_t* P, uint32_t M) {
  const uint32_t C = M - 1, NB = (C + R - 1) / R;
  const int H = (int)(M / 2);
  Sums s{0, 0, 0};
  for (uint32_t bi = 0; bi < NB; ++bi) {
    uint32_t xi[R][2];
    load_block2<NEED, R>(P, M, 1 + bi * R, xi);
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = a + 1; b < R; ++b)
        pair_step<NEED>(xi[a][0] ^ xi[b][0], xi[a][1] ^ xi[b][1], 2, H, s);
    for (uint32_t bj = bi + 1; bj < NB; ++bj) {
      uint32_t xj[R][2];
      load_block2<NEED, R>(P, M, 1 + bj * R, xj);
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b)
          pair_step<NEED>(xi[a][0] ^ xj[b][0], xi[a][1] ^ xj[b][1], 2, H, s);
    }
  }
  const uint32_t npad = NB * R - C, npp = npad * (npad - 1) / 2;
  s.sq -= npp * (uint32_t)(H * H);
  s.ab -= npp * (uint32_t)H;
  s.nz -= npp;
  return s;
}

__device__ __forceinline__ uint32_t key_of(uint32_t kind, const Sums& s) {
  switch (kind) {
    case kFitSQ: return 4u * s.sq;
    case kFitABS: return 2u * s.ab;
    case kFitNNZ: return s.nz;
    case kFitSQNNZ: return 4u * s.sq + s.nz;
    case kFitF1: return 4u * s.ab;   // sum_{i,j}|G| - m^2 = 2 * ABS
    default: return 2u * s.nz;       // nnz(G) - m = 2 * NNZ
  }
}

// Blocked pair sums of a memory-resident individual of runtime order
// 68 <= M <= 128 (four words per column), as blocked_sums_w2.
template <uint32_t NEED, int R>
__device__ __forceinline__ void load_block4(const uint32_t* P, uint32_t M,
                                            uint32_t col0, uint4 (&x)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t col = col0 + r;
    x[r] = col < M ? reinterpret_cast<const uint4*>(P)[col] : make_uint4(0, 0, 0, 0);
  }
}

template <uint32_t NEED, int R>
__device__ __forceinline__ Sums blocked_sums_w4(const uint32_t* P, uint32_t M) {
  const uint32_t C = M - 1, NB = (C + R - 1) / R;
  const int H = (int)(M / 2);
  Sums s{0, 0, 0};
  for (uint32_t bi = 0; bi < NB; ++bi) {
    uint4 xi[R];
    load_block4<NEED, R>(P, M, 1 + bi * R, xi);
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = a + 1; b < R; ++b) pair_step4<NEED, 4>(xi[a], xi[b], H, s);
    for (uint32_t bj = bi + 1; bj < NB; ++bj) {
      uint4 xj[R];
      load_block4<NEED, R>(P, M, 1 + bj * R, xj);
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) pair_step4<NEED, 4>(xi[a], xj[b], H, s);
    }
  }
  const uint32_t npad = NB * R - C, npp = npad * (npad - 1) / 2;
  s.sq -= npp * (uint32_t)(H * H);
  s.ab -= npp * (uint32_t)H;
  s.nz -= npp;
  return s;
}

template <uint32_t NEED>
__device__ __forceinline__ Sums sums_w2(const uint32_t* P, uint32_t M) {
  return M <= 44 ? blocked_sums_w2<NEED, 4>(P, M) : blocked_sums_w2<NEED, 8>(P, M);
}

// Key (and optionally the (SQ, ABS, NNZ) components) of one individual:
// register-resident (M <= 32) ...
template <int M>
__device__ __forceinline__ uint32_t fitness(const Cols<M>& c, uint32_t kind,
                                            bool comps, uint32_t* out3) {
  Sums s;
  if (comps) {
    s = pair_sums<M, kNeedSQ | kNeedABS | kNeedNNZ>(c);
  } else {
    switch (needs_of_kind(kind)) {
      case kNeedSQ: s = pair_sums<M, kNeedSQ>(c); break;
      case kNeedABS: s = pair_sums<M, kNeedABS>(c); break;
      case kNeedNNZ: s = pair_sums<M, kNeedNNZ>(c); break;
      default: s = pair_sums<M, kNeedSQ | kNeedNNZ>(c); break;
    }
  }
  if (comps) {
    out3[0] = 4u * s.sq;
    out3[1] = 2u * s.ab;
    out3[2] = s.nz;
  }
  return key_of(kind, s);
}

// ... or memory-resident, runtime order 36 <= M <= 64.
__device__ __forceinline__ uint32_t fitness_w2(const uint32_t* P, uint32_t M,
                                               uint32_t kind, bool comps,
                                               uint32_t* out3) {
  Sums s;
  if (comps) {
    s = sums_w2<kNeedSQ | kNeedABS | kNeedNNZ>(P, M);
  } else {
    switch (needs_of_kind(kind)) {
      case kNeedSQ: s = sums_w2<kNeedSQ>(P, M); break;
      case kNeedABS: s = sums_w2<kNeedABS>(P, M); break;
      case kNeedNNZ: s = sums_w2<kNeedNNZ>(P, M); break;
      default: s = sums_w2<kNeedSQ | kNeedNNZ>(P, M); break;
    }
  }
  if (comps) {
    out3[0] = 4u * s.sq;
    out3[1] = 2u * s.ab;
    out3[2] = s.nz;
  }
  return key_of(kind, s);
}

// ... or memory-resident, runtime order 68 <= M <= 128.
__device__ __forceinline__ uint32_t fitness_w4(const uint32_t* P, uint32_t M,
                                               uint32_t kind, bool comps,
                                               uint32_t* out3) {
  Sums s;
  if (comps) {
    s = blocked_sums_w4<kNeedSQ | kNeedABS | kNeedNNZ, 8>(P, M);
  } else {
    switch (needs_of_kind(kind)) {
      case kNeedSQ: s = blocked_sums_w4<kNeedSQ, 8>(P, M); break;
      case kNeedABS: s = blocked_sums_w4<kNeedABS, 8>(P, M); break;
      case kNeedNNZ: s = blocked_sums_w4<kNeedNNZ, 8>(P, M); break;
      default: s = blocked_sums_w4<kNeedSQ | kNeedNNZ, 8>(P, M); break;
    }
  }
  if (comps) {
    out3[0] = 4u * s.sq;
    out3[1] = 2u * s.ab;
    out3[2] = s.nz;
  }
  return key_of(kind, s);
}

// Load one packed individual (M*W words, a multiple of 4) with
// 16-byte accesses.
template <int M>
__device__ __forceinline__ void load_cols(const uint32_t* src, Cols<M>& c) {
  constexpr int W = Cols<M>::W;
  const uint4* s4 = reinterpret_cast<const uint4*>(src);
  uint32_t* flat = &c.w[0][0];
#pragma unroll
  for (int v = 0; v < M * W / 4; ++v) {
    const uint4 q = s4[v];
    flat[4 * v + 0] = q.x;
    flat[4 * v + 1] = q.y;
    flat[4 * v + 2] = q.z;
    flat[4 * v + 3] = q.w;
  }
}

// (a == J) ? x : 0, with the comparison kept opaque to the compiler: a
// column chosen at run time is then updated by a select per column instead
// of the indexed scratch access the compiler would otherwise emit.
template <int J>
__device__ __forceinline__ uint32_t pick_if_eq(uint32_t a, uint32_t x) {
  uint32_t r;
  asm("v_cmp_eq_u32 vcc, %2, %1\n\tv_cndmask_b32 %0, 0, %3, vcc"
      : "=v"(r)
      : "v"(a), "n"(J), "v"(x)
      : "vcc");
  return r;
}

}  // namespace ga
