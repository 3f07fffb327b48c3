/*
 * gao.c -- plain CPU oracle of the Hadamard-matrix genetic algorithm
 * (Balogh & Ruiz, arXiv 2208.14961).  TEST INFRASTRUCTURE ONLY: see gao.h.
 *
 * Everything here is written for a reader checking it against the paper:
 * int8 matrices with +1/-1 entries, a triple-loop Gram matrix, sequential
 * operators, qsort for ranking.  The only parallelism is an OpenMP loop over
 * independent individuals, which cannot change any result.
 */
#include "gao.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 3 and Table 2).                 */
/* Each round multiplies counter words 0 and 2 by two fixed odd constants,   */
/* swaps the halves of the products into the other words, xors in the round  */
/* key, and the key is bumped by two Weyl constants between rounds.          */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u /* golden ratio */
#define PHILOX_W1 0xBB67AE85u /* sqrt(3) - 1  */

void gao_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Draw number d of (stream, generation, index): word d%4 of the Philox block
 * whose counter is (d/4, index, generation, stream), keyed by the seed. */
uint32_t gao_draw(uint64_t seed, uint32_t stream, uint32_t gen, uint32_t idx,
                  uint32_t d) {
  uint32_t ctr[4] = {d / 4u, idx, gen, stream};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t out[4];
  gao_philox4x32_10(ctr, key, out);
  return out[d % 4u];
}

/* An integer in [0, range) from a 32-bit draw: floor(u * range / 2^32). */
uint32_t gao_bounded(uint32_t u, uint32_t range) {
  return (uint32_t)(((uint64_t)u * (uint64_t)range) >> 32);
}

static int bern(uint32_t u, uint64_t threshold) {
  return (uint64_t)u < threshold;
}

/* ------------------------------------------------------------------------ */
/* Configuration checks                                                      */
/* ------------------------------------------------------------------------ */
int gao_validate(const gao_config* c) {
  if (!c) return -1;
  if (c->m < 4 || c->m > GAO_MAX_M || c->m % 4 != 0) return -1;
  if (c->n < 2) return -1;
  if (c->fitness > GAO_FIT_F2) return -1;
  if (c->selection > GAO_SEL_PAPER) return -1;
  if (c->xo_threshold > (1ull << 32) || c->mut_threshold > (1ull << 32))
    return -1;
  if (c->nc > 64 || c->nr > 64) return -1;
  if (c->mut_threshold > 0 && (c->nc == 0 || c->nr == 0)) return -1;
  if (c->mut_shared > 1) return -1;
  if (c->selection == GAO_SEL_TOURNAMENT) {
    if (c->tournament_k < 1 || c->tournament_k > 64) return -1;
    if (c->elite >= c->n) return -1;
  } else {
    if (c->n % 4 != 0 || c->elite != 0) return -1;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Gram matrix and fitness (paper Sec. 3.2 and Sec. 4.2)                     */
/* ------------------------------------------------------------------------ */
void gao_gram(uint32_t m, const int8_t* Q, int32_t* G) {
  for (uint32_t i = 0; i < m; ++i)
    for (uint32_t j = 0; j < m; ++j) {
      int32_t s = 0;
      for (uint32_t r = 0; r < m; ++r)
        s += (int32_t)Q[r * m + i] * (int32_t)Q[r * m + j];
      G[i * m + j] = s;
    }
}

uint32_t gao_fitness_one(uint32_t m, uint32_t kind, const int8_t* Q,
                         uint32_t* comps) {
  int32_t G[GAO_MAX_M * GAO_MAX_M];
  gao_gram(m, Q, G);
  /* components over the pairs of distinct columns i < j */
  uint32_t sq = 0, ab = 0, nnz = 0;
  for (uint32_t i = 0; i < m; ++i)
    for (uint32_t j = i + 1; j < m; ++j) {
      int32_t g = G[i * m + j];
      sq += (uint32_t)(g * g);
      ab += (uint32_t)(g < 0 ? -g : g);
      nnz += (g != 0) ? 1u : 0u;
    }
  if (comps) {
    comps[0] = sq;
    comps[1] = ab;
    comps[2] = nnz;
  }
  switch (kind) {
    case GAO_FIT_SQ: return sq;
    case GAO_FIT_ABS: return ab;
    case GAO_FIT_NNZ: return nnz;
    case GAO_FIT_SQ_PLUS_NNZ: return sq + nnz;
    case GAO_FIT_F1: {
      /* Eq. (fitness0): sum of |entries| of Q^T Q over all (i, j), minus m^2 */
      int64_t s = 0;
      for (uint32_t i = 0; i < m * m; ++i) s += G[i] < 0 ? -G[i] : G[i];
      return (uint32_t)(s - (int64_t)m * m);
    }
    case GAO_FIT_F2: {
      /* Eq. (fitness): number of nonzero entries of Q^T Q, minus m */
      int64_t s = 0;
      for (uint32_t i = 0; i < m * m; ++i) s += G[i] != 0;
      return (uint32_t)(s - (int64_t)m);
    }
  }
  return 0xffffffffu;
}

int gao_fitness(const gao_config* c, const int8_t* pop, uint32_t* keys,
                uint32_t* comps) {
  if (gao_validate(c)) return -1;
  const uint32_t m = c->m;
  const int64_t n = c->n;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k)
    keys[k] = gao_fitness_one(m, c->fitness, pop + (size_t)k * m * m,
                              comps ? comps + 3 * k : NULL);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Initial population (paper Sec. 3.1): column 0 all +1; every other column  */
/* starts with its upper half -1 and lower half +1, then a Fisher-Yates      */
/* shuffle of that column.                                                   */
/* ------------------------------------------------------------------------ */
int gao_init_population(const gao_config* c, int8_t* pop) {
  if (gao_validate(c)) return -1;
  const uint32_t m = c->m;
  const int64_t n = c->n;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    int8_t* Q = pop + (size_t)k * m * m;
    for (uint32_t i = 0; i < m; ++i)
      for (uint32_t j = 0; j < m; ++j)
        Q[i * m + j] = (j > 0 && i < m / 2) ? -1 : 1;
    for (uint32_t j = 1; j < m; ++j)
      for (uint32_t i1 = 0; i1 + 1 < m; ++i1) {
        uint32_t u = gao_draw(c->seed, GAO_STREAM_INIT, 0, (uint32_t)k,
                              j * m + i1);
        uint32_t i2 = i1 + gao_bounded(u, m - i1);
        int8_t t = Q[i1 * m + j];
        Q[i1 * m + j] = Q[i2 * m + j];
        Q[i2 * m + j] = t;
      }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Crossover (paper Sec. 3.4): columns before the cut come from one parent,  */
/* the rest from the other; the second child takes the complement.          */
/* ------------------------------------------------------------------------ */
void gao_crossover(uint32_t m, const int8_t* A, const int8_t* B, uint32_t cut,
                   int8_t* O0, int8_t* O1) {
  for (uint32_t i = 0; i < m; ++i)
    for (uint32_t j = 0; j < m; ++j) {
      O0[i * m + j] = (j < cut) ? A[i * m + j] : B[i * m + j];
      O1[i * m + j] = (j < cut) ? B[i * m + j] : A[i * m + j];
    }
}

/* ------------------------------------------------------------------------ */
/* Mutation (paper Sec. 3.5, third method): for each chosen column, for each */
/* chosen row pair in turn, the two entries are negated only if they differ, */
/* which keeps the column balanced.                                          */
/* ------------------------------------------------------------------------ */
void gao_mutate(uint32_t m, int8_t* Q, uint32_t nc, const uint32_t* cols,
                uint32_t nr, const uint32_t* r1, const uint32_t* r2) {
  for (uint32_t jc = 0; jc < nc; ++jc) {
    uint32_t col = cols[jc];
    for (uint32_t ir = 0; ir < nr; ++ir) {
      int8_t* a = &Q[r1[ir] * m + col];
      int8_t* b = &Q[r2[ir] * m + col];
      if (*a != *b) {
        *a = (int8_t)-*a;
        *b = (int8_t)-*b;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Selection helpers                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t key, idx;
} key_idx;

static int cmp_key_idx(const void* pa, const void* pb) {
  const key_idx* a = (const key_idx*)pa;
  const key_idx* b = (const key_idx*)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
  return 0;
}

static int cmp_u32(const void* pa, const void* pb) {
  uint32_t a = *(const uint32_t*)pa, b = *(const uint32_t*)pb;
  return a < b ? -1 : (a > b ? 1 : 0);
}

void gao_select_set(const uint32_t* keys, uint32_t n, uint32_t count,
                    uint32_t* sel_out) {
  key_idx* v = (key_idx*)malloc(sizeof(key_idx) * n);
  for (uint32_t i = 0; i < n; ++i) {
    v[i].key = keys[i];
    v[i].idx = i;
  }
  qsort(v, n, sizeof(key_idx), cmp_key_idx);
  for (uint32_t s = 0; s < count; ++s) sel_out[s] = v[s].idx;
  qsort(sel_out, count, sizeof(uint32_t), cmp_u32);
  free(v);
}

/* A keyed pseudo-random permutation of [0, domain): a balanced eight-round
 * Feistel network on 2h bits (4^h >= domain) whose round function is a
 * Philox draw, restricted to [0, domain) by cycle-walking (repeat until the
 * value falls inside the domain; this ends because the cycle of the start
 * value returns to it). */
static uint32_t feistel(uint64_t seed, uint32_t gen, uint32_t h, uint32_t x) {
  uint32_t mask = (1u << h) - 1u;
  uint32_t L = x >> h, R = x & mask;
  for (uint32_t r = 0; r < 8; ++r) {
    uint32_t f = gao_draw(seed, GAO_STREAM_PERM, gen, R, r) & mask;
    uint32_t t = L ^ f;
    L = R;
    R = t;
  }
  return (L << h) | R;
}

uint32_t gao_permute(uint64_t seed, uint32_t gen, uint32_t domain,
                     uint32_t s) {
  uint32_t h = 1;
  while ((1ull << (2 * h)) < (uint64_t)domain) ++h;
  uint32_t x = s;
  do {
    x = feistel(seed, gen, h, x);
  } while (x >= domain);
  return x;
}

static int better(const uint32_t* keys, uint32_t x, uint32_t y) {
  return keys[x] < keys[y] || (keys[x] == keys[y] && x < y);
}

void gao_tournament_parents(const gao_config* c, const uint32_t* keys,
                            uint32_t gen_out, uint32_t p, uint32_t* a,
                            uint32_t* b) {
  uint32_t win[2];
  const uint32_t t = c->tournament_k;
  for (uint32_t s = 0; s < 2; ++s) {
    uint32_t best = 0;
    for (uint32_t k = 0; k < t; ++k) {
      uint32_t u = gao_draw(c->seed, GAO_STREAM_SELECT, gen_out, p, s * t + k);
      uint32_t x = gao_bounded(u, c->n);
      if (k == 0 || better(keys, x, best)) best = x;
    }
    win[s] = best;
  }
  *a = win[0];
  *b = win[1];
}

/* ------------------------------------------------------------------------ */
/* One generation: gen_in -> gen_in + 1                                      */
/* ------------------------------------------------------------------------ */
/* Crossover, mutation and evaluation of child pair p from parents A and B;
 * the children go to slots dst0 and dst1 (dst1 may be >= n: dropped). */
static void make_pair(const gao_config* c, uint32_t G, uint32_t p,
                      const int8_t* A, const int8_t* B, int8_t* pop_out,
                      uint32_t* keys_out, uint32_t dst0, uint32_t dst1) {
  const uint32_t m = c->m;
  int8_t O[2][GAO_MAX_M * GAO_MAX_M];
  if (bern(gao_draw(c->seed, GAO_STREAM_XOVER, G, p, 0), c->xo_threshold)) {
    uint32_t cut =
        1 + gao_bounded(gao_draw(c->seed, GAO_STREAM_XOVER, G, p, 1), m - 1);
    gao_crossover(m, A, B, cut, O[0], O[1]);
  } else {
    memcpy(O[0], A, (size_t)m * m);
    memcpy(O[1], B, (size_t)m * m);
  }
  const uint32_t dst[2] = {dst0, dst1};
  for (uint32_t ch = 0; ch < 2; ++ch) {
    if (dst[ch] >= c->n) continue;
    if (bern(gao_draw(c->seed, GAO_STREAM_XOVER, G, p, 2 + ch),
             c->mut_threshold)) {
      /* the child's own draws, or the generation's shared ones (first
       * mutation method, Sec. 3.5) */
      uint32_t q = c->mut_shared ? GAO_SHARED_MUTATION : 2 * p + ch;
      uint32_t cols[64], r1[64], r2[64];
      for (uint32_t jc = 0; jc < c->nc; ++jc)
        cols[jc] = 1 + gao_bounded(
                           gao_draw(c->seed, GAO_STREAM_MUTATE, G, q, jc),
                           m - 1);
      for (uint32_t ir = 0; ir < c->nr; ++ir) {
        r1[ir] = gao_bounded(
            gao_draw(c->seed, GAO_STREAM_MUTATE, G, q, c->nc + 2 * ir), m);
        r2[ir] = gao_bounded(
            gao_draw(c->seed, GAO_STREAM_MUTATE, G, q, c->nc + 2 * ir + 1),
            m);
      }
      gao_mutate(m, O[ch], c->nc, cols, c->nr, r1, r2);
    }
    memcpy(pop_out + (size_t)dst[ch] * m * m, O[ch], (size_t)m * m);
    keys_out[dst[ch]] = gao_fitness_one(m, c->fitness, O[ch], NULL);
  }
}

int gao_step(const gao_config* c, const int8_t* pop_in,
             const uint32_t* keys_in, int8_t* pop_out, uint32_t* keys_out,
             uint32_t gen_in) {
  if (gao_validate(c)) return -1;
  const uint32_t m = c->m, n = c->n, G = gen_in + 1;
  const size_t mm = (size_t)m * m;
  if (c->selection == GAO_SEL_TOURNAMENT) {
    const uint32_t e = c->elite;
    if (e > 0) {
      /* elites: the e smallest (key, index), kept in index order, unchanged */
      uint32_t* sel = (uint32_t*)malloc(sizeof(uint32_t) * e);
      gao_select_set(keys_in, n, e, sel);
      for (uint32_t s = 0; s < e; ++s) {
        memcpy(pop_out + s * mm, pop_in + (size_t)sel[s] * mm, mm);
        keys_out[s] = keys_in[sel[s]];
      }
      free(sel);
    }
    const int64_t pairs = (n - e + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < pairs; ++p) {
      uint32_t a, b;
      gao_tournament_parents(c, keys_in, G, (uint32_t)p, &a, &b);
      make_pair(c, G, (uint32_t)p, pop_in + (size_t)a * mm,
                pop_in + (size_t)b * mm, pop_out, keys_out,
                e + 2 * (uint32_t)p, e + 2 * (uint32_t)p + 1);
    }
  } else {
    /* paper mode (Sec. 3.3): the best 2N of the 4N matrices become the
     * parents, in random order; pair (P_k, P_{k+N}) makes O_k and O_{N+k} */
    const uint32_t N = n / 4, D = 2 * N;
    uint32_t* sel = (uint32_t*)malloc(sizeof(uint32_t) * D);
    gao_select_set(keys_in, n, D, sel);
    for (uint32_t s = 0; s < D; ++s) {
      uint32_t src = sel[gao_permute(c->seed, G, D, s)];
      memcpy(pop_out + s * mm, pop_in + (size_t)src * mm, mm);
      keys_out[s] = keys_in[src];
    }
    free(sel);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)N; ++k)
      make_pair(c, G, (uint32_t)k, pop_out + (size_t)k * mm,
                pop_out + (size_t)(k + N) * mm, pop_out, keys_out,
                2 * N + (uint32_t)k, 3 * N + (uint32_t)k);
  }
  return 0;
}

static void best_of(const uint32_t* keys, uint32_t n, uint32_t* idx,
                    uint32_t* key) {
  uint32_t b = 0;
  for (uint32_t i = 1; i < n; ++i)
    if (keys[i] < keys[b]) b = i;
  *idx = b;
  *key = keys[b];
}

int gao_run(const gao_config* c, int8_t* pop_final, uint32_t* keys_final,
            gao_result* res) {
  if (gao_validate(c)) return -1;
  const uint32_t n = c->n;
  const size_t bytes = (size_t)n * c->m * c->m;
  int8_t* pa = (int8_t*)malloc(bytes);
  int8_t* pb = (int8_t*)malloc(bytes);
  uint32_t* ka = (uint32_t*)malloc(sizeof(uint32_t) * n);
  uint32_t* kb = (uint32_t*)malloc(sizeof(uint32_t) * n);
  gao_init_population(c, pa);
  gao_fitness(c, pa, ka, NULL);
  uint32_t g = 0, bi, bk;
  best_of(ka, n, &bi, &bk);
  while (!(c->stop_on_found && bk == 0) && g < c->max_generations) {
    gao_step(c, pa, ka, pb, kb, g);
    ++g;
    int8_t* tp = pa; pa = pb; pb = tp;
    uint32_t* tk = ka; ka = kb; kb = tk;
    best_of(ka, n, &bi, &bk);
  }
  res->found = bk == 0;
  res->generation = g;
  res->index = bi;
  res->best_key = bk;
  if (pop_final) memcpy(pop_final, pa, bytes);
  if (keys_final) memcpy(keys_final, ka, sizeof(uint32_t) * n);
  free(pa); free(pb); free(ka); free(kb);
  return 0;
}

uint32_t gao_check_invariants(uint32_t m, uint32_t n, const int8_t* pop) {
  uint32_t bad = 0;
  for (uint32_t k = 0; k < n; ++k) {
    const int8_t* Q = pop + (size_t)k * m * m;
    int ok = 1;
    for (uint32_t i = 0; i < m; ++i) ok &= Q[i * m] == 1;
    for (uint32_t j = 1; j < m; ++j) {
      uint32_t minus = 0;
      for (uint32_t i = 0; i < m; ++i) {
        ok &= (Q[i * m + j] == 1 || Q[i * m + j] == -1);
        minus += Q[i * m + j] == -1;
      }
      ok &= minus == m / 2;
    }
    bad += !ok;
  }
  return bad;
}

int gao_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void gao_set_num_threads(int threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
}
