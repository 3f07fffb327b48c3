// ga_kernels.hip -- initialization, standalone fitness, run-state and
// invariant-check kernels of libga (gfx950) and their launchers.
//
// One lane per individual.  A lane keeps the packed columns of its matrix
// in registers (orders up to 32) or reads them in register tiles (orders
// 36..128), so the Gram matrix is never materialized: each off-diagonal
// entry is one xor and one popcount per word, reduced into the key on the
// fly.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ga_common.h"
#include "ga_device.h"

namespace ga {

// ---------------------------------------------------------------------------
// Initial population (Sec. 3.1): one thread per (matrix k, column j).
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kBlock) void init_kernel(uint32_t* pop,
                                                      uint32_t n,
                                                      uint64_t seed) {
  constexpr int W = (int)col_words(M);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint64_t)n * M) return;
  const uint32_t k = (uint32_t)(t / M), j = (uint32_t)(t % M);
  if constexpr (M > 64) {
    // rows 0..127 as two 64-bit halves
    uint64_t lo = 0, hi = 0;
    if (j > 0) {
      lo = (M / 2 == 64) ? ~0ull : ((1ull << (M / 2)) - 1ull);
#pragma unroll
      for (int b = 0; b < M / 4; ++b) {
        const U4 u = draw_block(seed, kStreamInit, 0, k, j * (M / 4) + b);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int i1 = 4 * b + w;
          if (i1 >= M - 1) break;
          const uint32_t i2 = (uint32_t)i1 + bounded(u[w], (uint32_t)(M - i1));
          const uint64_t b1 = i1 < 64 ? (lo >> i1) & 1ull : (hi >> (i1 - 64)) & 1ull;
          const uint64_t b2 = i2 < 64 ? (lo >> i2) & 1ull : (hi >> (i2 - 64)) & 1ull;
          if (b1 != b2) {
            if (i1 < 64) lo ^= 1ull << i1; else hi ^= 1ull << (i1 - 64);
            if (i2 < 64) lo ^= 1ull << i2; else hi ^= 1ull << (i2 - 64);
          }
        }
      }
    }
    reinterpret_cast<uint4*>(pop)[(size_t)k * M + j] =
        make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
  } else {
    uint64_t v = 0;
    if (j > 0) {
      v = (M / 2 == 64) ? ~0ull : ((1ull << (M / 2)) - 1ull);  // rows < M/2 = -1
      // Fisher-Yates over rows: draws d = j*M + i1 are whole blocks j*M/4 ...
#pragma unroll
      for (int b = 0; b < M / 4; ++b) {
        const U4 u = draw_block(seed, kStreamInit, 0, k, j * (M / 4) + b);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int i1 = 4 * b + w;
          if (i1 >= M - 1) break;
          const uint32_t i2 = (uint32_t)i1 + bounded(u[w], (uint32_t)(M - i1));
          const uint64_t b1 = (v >> i1) & 1ull, b2 = (v >> i2) & 1ull;
          if (b1 != b2) v ^= (1ull << i1) | (1ull << i2);
        }
      }
    }
    uint32_t* dst = pop + ((size_t)k * M + j) * W;
    dst[0] = (uint32_t)v;
    if (W > 1) dst[1] = (uint32_t)(v >> 32);
  }
}

// ---------------------------------------------------------------------------
// Standalone fitness (Sec. 3.2): one lane per individual.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fitness_epilogue(uint32_t k, uint32_t key,
                                                 const uint32_t* out3,
                                                 uint32_t* keys, uint32_t* comps,
                                                 unsigned long long* best) {
  keys[k] = key;
  if (comps) {
    comps[3 * (size_t)k + 0] = out3[0];
    comps[3 * (size_t)k + 1] = out3[1];
    comps[3 * (size_t)k + 2] = out3[2];
  }
  *best = ((unsigned long long)key << 32) | k;
}

template <int M>
__global__ __launch_bounds__(kChildBlock) void fitness_kernel(
    const uint32_t* __restrict__ pop, uint32_t n, uint32_t kind,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ comps, RunState* st) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long best = ~0ull;
  if (k < n) {
    Cols<M> c;
    load_cols<M>(pop + (size_t)k * M, c);
    uint32_t out3[3];
    const uint32_t key = fitness<M>(c, kind, comps != nullptr, out3);
    fitness_epilogue(k, key, out3, keys, comps, &best);
  }
  if (st) note_zero(st, best, 0);
}

__global__ __launch_bounds__(kChildBlock) void fitness_kernel_w2(
    const uint32_t* __restrict__ pop, uint32_t n, uint32_t m, uint32_t kind,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ comps, RunState* st) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long best = ~0ull;
  if (k < n) {
    uint32_t out3[3];
    const uint32_t key =
        fitness_w2(pop + (size_t)k * 2 * m, m, kind, comps != nullptr, out3);
    fitness_epilogue(k, key, out3, keys, comps, &best);
  }
  if (st) note_zero(st, best, 0);
}

__global__ __launch_bounds__(kChildBlock) void fitness_kernel_w4(
    const uint32_t* __restrict__ pop, uint32_t n, uint32_t m, uint32_t kind,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ comps, RunState* st) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long best = ~0ull;
  if (k < n) {
    uint32_t out3[3];
    const uint32_t key =
        fitness_w4(pop + (size_t)k * 4 * m, m, kind, comps != nullptr, out3);
    fitness_epilogue(k, key, out3, keys, comps, &best);
  }
  if (st) note_zero(st, best, 0);
}

// ga_fitness_repeat: evaluation i of the launch is individual i mod n, for
// i < n * reps, strided over a grid sized to fill every CU.
template <int M, uint32_t NEED>
__global__ __launch_bounds__(kBlock) void fitness_repeat_kernel(
    const uint32_t* __restrict__ pop, uint32_t n, uint64_t total, uint32_t kind,
    uint32_t* __restrict__ keys) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t k = (uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) % n);
  const uint32_t step = (uint32_t)(stride % n);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += stride) {
    Cols<M> c;
    load_cols<M>(pop + (size_t)k * M, c);
    keys[k] = key_of(kind, pair_sums<M, NEED>(c));
    k += step;
    k = k >= n ? k - n : k;
  }
}

__global__ __launch_bounds__(kBlock) void fitness_repeat_w2_kernel(
    const uint32_t* __restrict__ pop, uint32_t n, uint32_t m, uint64_t total,
    uint32_t kind, uint32_t* __restrict__ keys) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t k = (uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) % n);
  const uint32_t step = (uint32_t)(stride % n);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += stride) {
    keys[k] = fitness_w2(pop + (size_t)k * 2 * m, m, kind, false, nullptr);
    k += step;
    k = k >= n ? k - n : k;
  }
}

__global__ __launch_bounds__(kBlock) void fitness_repeat_w4_kernel(
    const uint32_t* __restrict__ pop, uint32_t n, uint32_t m, uint64_t total,
    uint32_t kind, uint32_t* __restrict__ keys) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t k = (uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) % n);
  const uint32_t step = (uint32_t)(stride % n);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += stride) {
    keys[k] = fitness_w4(pop + (size_t)k * 4 * m, m, kind, false, nullptr);
    k += step;
    k = k >= n ? k - n : k;
  }
}

__global__ void reset_state_kernel(RunState* st) {
  st->best = ~0ull;
  st->gen_base = 0;
  st->found_gen = ~0u;
  st->final_gen = 0;
}

__global__ void set_state_kernel(RunState* st, uint32_t gen) {
  st->best = ~0ull;
  st->gen_base = gen;
  st->found_gen = ~0u;
  st->final_gen = gen + 1;
}

// gen_base += k for the runs of a launch table (one thread per run) or one
// run.
__global__ void advance_kernel(const PopDesc* __restrict__ descs, uint32_t ndesc,
                               uint32_t k) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ndesc) descs[i].state->gen_base += k;
}

__global__ void advance_one_kernel(RunState* st, uint32_t k) {
  st->gen_base += k;
}

// The reported generation of a run (the first one holding a key of 0 when
// stopping on a solution, else the last one) and its best (key, slot), the
// lowest slot among equal keys.  One block per run.
__device__ __forceinline__ void finish_run(const PopDesc& d) {
  RunState* st = d.state;
  const uint32_t found = st->found_gen;
  const uint32_t g = (d.stop_on_found && found <= d.max_gen) ? found : d.max_gen;
  const uint32_t* keys = (g & 1u) ? d.keys_b : d.keys_a;
  unsigned long long best = ~0ull;
  for (uint32_t i = threadIdx.x; i < d.n; i += kBlock) {
    const unsigned long long v = ((unsigned long long)keys[i] << 32) | i;
    best = v < best ? v : best;
  }
  best = block_min_u64(best);
  if (threadIdx.x == 0) {
    st->best = best;
    st->final_gen = g;
  }
}

__global__ __launch_bounds__(kBlock) void finish_kernel(
    const PopDesc* __restrict__ descs) {
  finish_run(descs[blockIdx.x]);
}

// The same for one run over several blocks: each block's smallest (key,
// slot) meets the others in one 64-bit atomic minimum (the state's best is
// ~0 from the run's start).
__global__ __launch_bounds__(kBlock) void finish_one_kernel(PopDesc d) {
  RunState* st = d.state;
  const uint32_t found = st->found_gen;
  const uint32_t g = (d.stop_on_found && found <= d.max_gen) ? found : d.max_gen;
  const uint32_t* keys = (g & 1u) ? d.keys_b : d.keys_a;
  unsigned long long best = ~0ull;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < d.n; i += gridDim.x * kBlock) {
    const unsigned long long v = ((unsigned long long)keys[i] << 32) | i;
    best = v < best ? v : best;
  }
  best = block_min_u64(best);
  if (threadIdx.x == 0) {
    atomicMin(&st->best, best);
    if (blockIdx.x == 0) st->final_gen = g;
  }
}

// ---------------------------------------------------------------------------
// Invariant check: column 0 zero, other columns balanced, no bits >= m.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void check_kernel(const uint32_t* pop,
                                                       uint32_t n, uint32_t m,
                                                       uint32_t* bad) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t W = col_words(m);
  const uint32_t* Q = pop + (size_t)k * m * W;
  bool ok = true;
  for (uint32_t w = 0; w < W; ++w) ok &= Q[w] == 0;
  for (uint32_t j = 1; j < m; ++j) {
    uint32_t pc = 0;
    for (uint32_t w = 0; w < W; ++w) {
      const uint32_t x = Q[j * W + w];
      const uint32_t rows = (m > 32 * w) ? min(32u, m - 32 * w) : 0u;
      const uint32_t valid = rows == 32 ? 0xffffffffu : ((1u << rows) - 1u);
      ok &= (x & ~valid) == 0;
      pc += __popc(x);
    }
    ok &= pc == m / 2;
  }
  if (!ok) atomicAdd(bad, 1u);
}

// ---------------------------------------------------------------------------
// Layout conversion: one thread per (matrix k, column j); the threads of a
// matrix touch consecutive bytes of each row.
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kBlock) void pack_kernel(const int8_t* __restrict__ q,
                                                      uint32_t* __restrict__ pop,
                                                      uint32_t n, uint32_t* bad) {
  constexpr int W = (int)col_words(M);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint64_t)n * M) return;
  const uint32_t k = (uint32_t)(t / M), j = (uint32_t)(t % M);
  const int8_t* src = q + (size_t)k * M * M + j;
  uint32_t w[4] = {0, 0, 0, 0};
  uint32_t odd = 0;
#pragma unroll
  for (int r = 0; r < M; ++r) {
    const int8_t e = src[(size_t)r * M];
    w[r / 32] |= (e < 0 ? 1u : 0u) << (r % 32);
    odd += (e != 1 && e != -1) ? 1u : 0u;
  }
  uint32_t* dst = pop + ((size_t)k * M + j) * W;
#pragma unroll
  for (int i = 0; i < W; ++i) dst[i] = w[i];
  if (odd && bad) atomicAdd(bad, odd);
}

template <int M>
__global__ __launch_bounds__(kBlock) void unpack_kernel(const uint32_t* __restrict__ pop,
                                                        int8_t* __restrict__ q, uint32_t n) {
  constexpr int W = (int)col_words(M);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (uint64_t)n * M) return;
  const uint32_t k = (uint32_t)(t / M), j = (uint32_t)(t % M);
  const uint32_t* src = pop + ((size_t)k * M + j) * W;
  uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = src[i];
  int8_t* dst = q + (size_t)k * M * M + j;
#pragma unroll
  for (int r = 0; r < M; ++r)
    dst[(size_t)r * M] = ((w[r / 32] >> (r % 32)) & 1u) ? (int8_t)-1 : (int8_t)1;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define GA_DISPATCH_M(m, EXPR)                  \
  switch (m) {                                  \
    case 4: { constexpr int MM = 4; EXPR; } break;   \
    case 8: { constexpr int MM = 8; EXPR; } break;   \
    case 12: { constexpr int MM = 12; EXPR; } break; \
    case 16: { constexpr int MM = 16; EXPR; } break; \
    case 20: { constexpr int MM = 20; EXPR; } break; \
    case 24: { constexpr int MM = 24; EXPR; } break; \
    case 28: { constexpr int MM = 28; EXPR; } break; \
    case 32: { constexpr int MM = 32; EXPR; } break; \
    case 36: { constexpr int MM = 36; EXPR; } break; \
    case 40: { constexpr int MM = 40; EXPR; } break; \
    case 44: { constexpr int MM = 44; EXPR; } break; \
    case 48: { constexpr int MM = 48; EXPR; } break; \
    case 52: { constexpr int MM = 52; EXPR; } break; \
    case 56: { constexpr int MM = 56; EXPR; } break; \
    case 60: { constexpr int MM = 60; EXPR; } break; \
    case 64: { constexpr int MM = 64; EXPR; } break; \
    case 68: { constexpr int MM = 68; EXPR; } break; \
    case 72: { constexpr int MM = 72; EXPR; } break; \
    case 76: { constexpr int MM = 76; EXPR; } break; \
    case 80: { constexpr int MM = 80; EXPR; } break; \
    case 84: { constexpr int MM = 84; EXPR; } break; \
    case 88: { constexpr int MM = 88; EXPR; } break; \
    case 92: { constexpr int MM = 92; EXPR; } break; \
    case 96: { constexpr int MM = 96; EXPR; } break; \
    case 100: { constexpr int MM = 100; EXPR; } break; \
    case 104: { constexpr int MM = 104; EXPR; } break; \
    case 108: { constexpr int MM = 108; EXPR; } break; \
    case 112: { constexpr int MM = 112; EXPR; } break; \
    case 116: { constexpr int MM = 116; EXPR; } break; \
    case 120: { constexpr int MM = 120; EXPR; } break; \
    case 124: { constexpr int MM = 124; EXPR; } break; \
    case 128: { constexpr int MM = 128; EXPR; } break; \
    default: return hipErrorInvalidValue;       \
  }

hipError_t launch_init(const ga_config* c, uint32_t* pop, hipStream_t s) {
  const uint32_t grid = cdiv((uint64_t)c->n * c->m, kBlock);
  GA_DISPATCH_M(c->m, hipLaunchKernelGGL(init_kernel<MM>, dim3(grid),
                                         dim3(kBlock), 0, s, pop, c->n,
                                         c->seed));
  return hipGetLastError();
}

hipError_t launch_pack(const ga_config* c, const int8_t* q, uint32_t* pop, uint32_t* bad,
                       hipStream_t s) {
  const uint32_t grid = cdiv((uint64_t)c->n * c->m, kBlock);
  GA_DISPATCH_M(c->m, hipLaunchKernelGGL(pack_kernel<MM>, dim3(grid), dim3(kBlock), 0, s, q,
                                         pop, c->n, bad));
  return hipGetLastError();
}

hipError_t launch_unpack(const ga_config* c, const uint32_t* pop, int8_t* q, hipStream_t s) {
  const uint32_t grid = cdiv((uint64_t)c->n * c->m, kBlock);
  GA_DISPATCH_M(c->m, hipLaunchKernelGGL(unpack_kernel<MM>, dim3(grid), dim3(kBlock), 0, s,
                                         pop, q, c->n));
  return hipGetLastError();
}

hipError_t launch_fitness(const ga_config* c, const uint32_t* pop,
                          uint32_t* keys, uint32_t* comps, RunState* st,
                          hipStream_t s) {
  // (the MFMA grid's cap: eight workgroups per CU of the 256 of an MI355X)
  if (use_mfma(c)) return launch_fitness_mfma(c, pop, keys, comps, st, c->n, 256, s);
  const uint32_t grid = cdiv(c->n, kChildBlock);
  if (c->m > 64) {
    hipLaunchKernelGGL(fitness_kernel_w4, dim3(grid), dim3(kChildBlock), 0, s, pop,
                       c->n, c->m, c->fitness, keys, comps, st);
    return hipGetLastError();
  }
  if (c->m > 32) {
    hipLaunchKernelGGL(fitness_kernel_w2, dim3(grid), dim3(kChildBlock), 0, s, pop,
                       c->n, c->m, c->fitness, keys, comps, st);
    return hipGetLastError();
  }
  switch (c->m) {
#define GA_FIT_CASE(MM)                                                       \
  case MM:                                                                    \
    hipLaunchKernelGGL(fitness_kernel<MM>, dim3(grid), dim3(kChildBlock), 0, s, \
                       pop, c->n, c->fitness, keys, comps, st);              \
    break;
    GA_FIT_CASE(4) GA_FIT_CASE(8) GA_FIT_CASE(12) GA_FIT_CASE(16)
    GA_FIT_CASE(20) GA_FIT_CASE(24) GA_FIT_CASE(28) GA_FIT_CASE(32)
#undef GA_FIT_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fitness_repeat(const ga_config* c, const uint32_t* pop,
                                 uint32_t* keys, uint32_t reps, uint32_t cus,
                                 hipStream_t s) {
  const uint64_t total = (uint64_t)c->n * reps;
  if (use_mfma(c)) return launch_fitness_mfma(c, pop, keys, nullptr, nullptr, total, cus, s);
  // eight workgroups of four waves per CU, fewer if the work is smaller
  const uint64_t grid = std::min<uint64_t>((uint64_t)cus * 8, cdiv(total, kBlock));
  if (c->m > 64) {
    hipLaunchKernelGGL(fitness_repeat_w4_kernel, dim3((uint32_t)grid), dim3(kBlock), 0, s,
                       pop, c->n, c->m, total, c->fitness, keys);
    return hipGetLastError();
  }
  if (c->m > 32) {
    hipLaunchKernelGGL(fitness_repeat_w2_kernel, dim3((uint32_t)grid), dim3(kBlock), 0, s,
                       pop, c->n, c->m, total, c->fitness, keys);
    return hipGetLastError();
  }
  const uint32_t need = needs_of_kind(c->fitness);
  switch (c->m) {
#define GA_REP_NEED(MM, NN)                                                     \
  hipLaunchKernelGGL((fitness_repeat_kernel<MM, NN>), dim3((uint32_t)grid),     \
                     dim3(kBlock), 0, s, pop, c->n, total, c->fitness, keys)
#define GA_REP_CASE(MM)                                                         \
  case MM:                                                                      \
    if (need == kNeedSQ) GA_REP_NEED(MM, kNeedSQ);                              \
    else if (need == kNeedABS) GA_REP_NEED(MM, kNeedABS);                       \
    else if (need == kNeedNNZ) GA_REP_NEED(MM, kNeedNNZ);                       \
    else GA_REP_NEED(MM, kNeedSQ | kNeedNNZ);                                   \
    break;
    GA_REP_CASE(4) GA_REP_CASE(8) GA_REP_CASE(12) GA_REP_CASE(16)
    GA_REP_CASE(20) GA_REP_CASE(24) GA_REP_CASE(28) GA_REP_CASE(32)
#undef GA_REP_NEED
#undef GA_REP_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reset_state(RunState* st, hipStream_t s) {
  hipLaunchKernelGGL(reset_state_kernel, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_set_state(RunState* st, uint32_t gen, hipStream_t s) {
  hipLaunchKernelGGL(set_state_kernel, dim3(1), dim3(1), 0, s, st, gen);
  return hipGetLastError();
}

hipError_t launch_advance(const PopDesc* descs_dev, uint32_t ndesc, uint32_t k,
                          hipStream_t s) {
  if (ndesc == 0) return hipSuccess;
  hipLaunchKernelGGL(advance_kernel, dim3(cdiv(ndesc, kBlock)), dim3(kBlock),
                     0, s, descs_dev, ndesc, k);
  return hipGetLastError();
}

hipError_t launch_advance_one(RunState* st, uint32_t k, hipStream_t s) {
  hipLaunchKernelGGL(advance_one_kernel, dim3(1), dim3(1), 0, s, st, k);
  return hipGetLastError();
}

hipError_t launch_finish(const PopDesc* descs_dev, uint32_t ndesc,
                         hipStream_t s) {
  if (ndesc == 0) return hipSuccess;
  hipLaunchKernelGGL(finish_kernel, dim3(ndesc), dim3(kBlock), 0, s, descs_dev);
  return hipGetLastError();
}

hipError_t launch_finish_one(const PopDesc& d, hipStream_t s) {
  // about eight keys per thread, at most 512 blocks
  const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(512, cdiv(d.n, 8 * kBlock)));
  hipLaunchKernelGGL(finish_one_kernel, dim3(blocks), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_check(const ga_config* c, const uint32_t* pop, uint32_t* bad,
                        hipStream_t s) {
  hipLaunchKernelGGL(check_kernel, dim3(cdiv(c->n, kBlock)), dim3(kBlock), 0,
                     s, pop, c->n, c->m, bad);
  return hipGetLastError();
}

}  // namespace ga
