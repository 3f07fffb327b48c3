// ga_mfma.hip -- the Gram + fitness of ga_fitness and ga_fitness_repeat on
// the matrix cores (int8 MFMA with int32 accumulation), orders 36..128.
//
// With x the 0/1 indicator of the -1 entries (the packed bits), the Gram
// entry of balanced columns i, j >= 1 is G_ij = m - 2 popcount(x_i ^ x_j)
// = 4 s_ij - m with s_ij = sum_r x_ri x_rj (Sec. 3.2, on bits): S = X^T X is
// a dense contraction over the m rows.  One wave computes one individual's
// S in 16 x 16 tiles with v_mfma_i32_16x16x64_i8 (rows in steps of 64; rows
// past m and columns past m - 1 are zero bytes), upper-triangle tiles only,
// and reduces d = m/2 - 2 s_ij = -G_ij / 2 over the pairs 1 <= i < j < m
// into the same (SQ, ABS, NNZ) sums as the popcount path.
//
// No entry is masked.  Column 0 and the padding columns are zero, so every
// entry involving one has s = 0, d = m/2; every diagonal entry of a balanced
// column has d = -m/2.  Each sum's term f(d) (d^2, |d|, [d != 0]) is the
// same for both, so the unwanted entries add a known count times f(m/2).
// The diagonal tiles hold each of their pairs twice (once per triangle):
// with D and O the sums over diagonal and off-diagonal tiles, the pairs sum
// to (O - n_off f(m/2)) + (D - n_diag f(m/2)) / 2, the counts coming from
// the host (mfma_counts).
//
// Operands.  For tile t and row step ks, lane l holds the 16 bytes of
// column c = 16 t + (l mod 16), rows 64 ks + 16 (l / 16) .. + 15: four
// groups of 4 bits spread into bytes by one 24-bit multiply each.  The same
// registers are the A operand (rows of X^T) of row tile t and the B operand
// (columns of X) of column tile t.  The instruction's output holds S[i][j]
// of the tile in lane l, register r with i = 4 (l / 16) + r, j = l mod 16.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ga_common.h"
#include "ga_device.h"

namespace ga {

typedef int v4i __attribute__((ext_vector_type(4)));

// Bits 0..3 of x into the low bit of bytes 0..3: the shifted copies of x at
// 0, 7, 14 and 21 bits do not overlap, so the product is their union.
__device__ __forceinline__ int spread4(uint32_t x) {
  return (int)(__umul24(x & 15u, 0x204081u) & 0x01010101u);
}

// The operand registers of one individual: T column tiles, KS row steps.
template <int T, int KS>
struct MfmaOps {
  v4i op[T][KS];
};

// Loads and spreads the operands of the individual at P (order M, W words
// per column, W = 2 KS).
template <int T, int KS>
__device__ __forceinline__ void mfma_load(const uint32_t* P, uint32_t M, MfmaOps<T, KS>& o) {
  constexpr int W = 2 * KS;
  const uint32_t l = threadIdx.x & 63u, c0 = l & 15u, g = l >> 4;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const uint32_t c = 16u * t + c0;
    uint32_t w[W];
    if constexpr (W == 2) {
      const uint2 v = c < M ? reinterpret_cast<const uint2*>(P)[c] : make_uint2(0, 0);
      w[0] = v.x;
      w[1] = v.y;
    } else {
      const uint4 v = c < M ? reinterpret_cast<const uint4*>(P)[c] : make_uint4(0, 0, 0, 0);
      w[0] = v.x;
      w[1] = v.y;
      w[2] = v.z;
      w[3] = v.w;
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      // rows 64 ks + 16 g .. + 15: half (g & 1) of word 2 ks + g / 2
      const uint32_t lo = w[2 * ks], hi = w[2 * ks + 1];
      const uint32_t word = (g >> 1) ? hi : lo;
      const uint32_t b = (g & 1u) ? word >> 16 : word & 0xFFFFu;
      o.op[t][ks] = v4i{spread4(b), spread4(b >> 4), spread4(b >> 8), spread4(b >> 12)};
    }
  }
}

// This lane's share of the sums over every entry of the diagonal tiles
// (*dg) and of the tiles above them (*of).
template <uint32_t NEED>
__device__ __forceinline__ void add_tile(const v4i& acc, int H, Sums& s) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int d = H - 2 * acc[r];
    if (NEED & kNeedSQ) s.sq = acc_sq(s.sq, d);
    if (NEED & kNeedABS) s.ab = acc_abs(s.ab, (uint32_t)(d + H), (uint32_t)H);
    if (NEED & kNeedNNZ) s.nz = acc_nz(s.nz, d);
  }
}
template <int T, int KS, uint32_t NEED>
__device__ __forceinline__ void mfma_tile_sums(const MfmaOps<T, KS>& o, uint32_t M, Sums* dg,
                                               Sums* of) {
  const int H = (int)(M / 2);
  *dg = Sums{0, 0, 0};
  *of = Sums{0, 0, 0};
#pragma unroll
  for (int ti = 0; ti < T; ++ti) {
#pragma unroll
    for (int tj = ti; tj < T; ++tj) {
      v4i acc = {0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.op[ti][ks], o.op[tj][ks], acc, 0, 0, 0);
      add_tile<NEED>(acc, H, tj == ti ? *dg : *of);
    }
  }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off, 64);
  return v;
}

// The pair sums of the individual at P, in every lane.  n_diag, n_off: the
// unwanted entries of the diagonal and the off-diagonal tiles.
template <int T, int KS, uint32_t NEED>
__device__ __forceinline__ Sums mfma_sums(const uint32_t* P, uint32_t M, uint32_t n_diag,
                                          uint32_t n_off) {
  MfmaOps<T, KS> o;
  mfma_load<T, KS>(P, M, o);
  Sums dg, of;
  mfma_tile_sums<T, KS, NEED>(o, M, &dg, &of);
  const uint32_t H = M / 2;
  Sums s{0, 0, 0};
  if (NEED & kNeedSQ)
    s.sq = (wave_sum(of.sq) - n_off * H * H) + (wave_sum(dg.sq) - n_diag * H * H) / 2;
  if (NEED & kNeedABS)
    s.ab = (wave_sum(of.ab) - n_off * H) + (wave_sum(dg.ab) - n_diag * H) / 2;
  if (NEED & kNeedNNZ) s.nz = (wave_sum(of.nz) - n_off) + (wave_sum(dg.nz) - n_diag) / 2;
  return s;
}

// Evaluation e of the launch is individual e mod n, for e < total; one wave
// per evaluation, strided over the grid.  comps (with NEED = all three
// sums) and st as in ga_fitness; st non-null only when total == n.
template <int T, int KS, uint32_t NEED>
__global__ __launch_bounds__(kBlock) void fitness_mfma_kernel(
    const uint32_t* __restrict__ pop, uint32_t n, uint32_t m, uint64_t total, uint32_t kind,
    uint32_t n_diag, uint32_t n_off, uint32_t* __restrict__ keys, uint32_t* __restrict__ comps,
    RunState* st) {
  constexpr uint32_t kWaves = kBlock / 64;
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t stride = (uint64_t)gridDim.x * kWaves;
  const size_t words = (size_t)m * 2 * KS;
  for (uint64_t e = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); e < total; e += stride) {
    const uint32_t k = (uint32_t)(e % n);
    const Sums s = mfma_sums<T, KS, NEED>(pop + k * words, m, n_diag, n_off);
    const uint32_t key = key_of(kind, s);
    if (lane == 0) {
      keys[k] = key;
      if (comps) {  // (SQ, ABS, NNZ)
        comps[3 * (size_t)k + 0] = 4u * s.sq;
        comps[3 * (size_t)k + 1] = 2u * s.ab;
        comps[3 * (size_t)k + 2] = s.nz;
      }
    }
    if (st) note_zero(st, lane == 0 ? ((unsigned long long)key << 32) | k : ~0ull, 0);
  }
}

// The entries of the tiles that are not pairs 1 <= i < j < m: in the
// diagonal tiles every entry but the pairs (counted in both triangles), in
// the tiles above them those in row 0 or in a padding column.
static void mfma_counts(uint32_t m, uint32_t T, uint32_t* n_diag, uint32_t* n_off) {
  uint32_t nd = 0, no = 0;
  for (uint32_t i = 0; i < 16 * T; ++i)
    for (uint32_t j = 0; j < 16 * T; ++j) {
      const bool pair = i >= 1 && j >= 1 && i < m && j < m && i != j;
      if (i / 16 == j / 16) nd += pair ? 0u : 1u;
      else if (i / 16 < j / 16) no += pair ? 0u : 1u;
    }
  *n_diag = nd;
  *n_off = no;
}

template <int T, int KS>
static hipError_t launch_mfma_tiles(const ga_config* c, const uint32_t* pop, uint32_t* keys,
                                    uint32_t* comps, RunState* st, uint64_t total, uint32_t grid,
                                    hipStream_t s) {
  const dim3 g(grid), b(kBlock);
  uint32_t nd, no;
  mfma_counts(c->m, T, &nd, &no);
  if (comps) {
    hipLaunchKernelGGL((fitness_mfma_kernel<T, KS, kNeedSQ | kNeedABS | kNeedNNZ>), g, b, 0, s,
                       pop, c->n, c->m, total, c->fitness, nd, no, keys, comps, st);
    return hipGetLastError();
  }
  switch (needs_of_kind(c->fitness)) {
    case kNeedSQ:
      hipLaunchKernelGGL((fitness_mfma_kernel<T, KS, kNeedSQ>), g, b, 0, s, pop, c->n, c->m,
                         total, c->fitness, nd, no, keys, comps, st);
      break;
    case kNeedABS:
      hipLaunchKernelGGL((fitness_mfma_kernel<T, KS, kNeedABS>), g, b, 0, s, pop, c->n, c->m,
                         total, c->fitness, nd, no, keys, comps, st);
      break;
    case kNeedNNZ:
      hipLaunchKernelGGL((fitness_mfma_kernel<T, KS, kNeedNNZ>), g, b, 0, s, pop, c->n, c->m,
                         total, c->fitness, nd, no, keys, comps, st);
      break;
    default:
      hipLaunchKernelGGL((fitness_mfma_kernel<T, KS, kNeedSQ | kNeedNNZ>), g, b, 0, s, pop,
                         c->n, c->m, total, c->fitness, nd, no, keys, comps, st);
  }
  return hipGetLastError();
}

hipError_t launch_fitness_mfma(const ga_config* c, const uint32_t* pop, uint32_t* keys,
                               uint32_t* comps, RunState* st, uint64_t total, uint32_t cus,
                               hipStream_t s) {
  // one wave per evaluation, at most eight workgroups of four waves per CU
  const uint32_t waves = kBlock / 64;
  const uint32_t grid =
      (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)cus * 8, (total + waves - 1) / waves));
  const uint32_t T = (c->m + 15) / 16;
  if (c->m <= 64) {
    switch (T) {
      case 3: return launch_mfma_tiles<3, 1>(c, pop, keys, comps, st, total, grid, s);
      case 4: return launch_mfma_tiles<4, 1>(c, pop, keys, comps, st, total, grid, s);
    }
  } else {
    switch (T) {
      case 5: return launch_mfma_tiles<5, 2>(c, pop, keys, comps, st, total, grid, s);
      case 6: return launch_mfma_tiles<6, 2>(c, pop, keys, comps, st, total, grid, s);
      case 7: return launch_mfma_tiles<7, 2>(c, pop, keys, comps, st, total, grid, s);
      case 8: return launch_mfma_tiles<8, 2>(c, pop, keys, comps, st, total, grid, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace ga
