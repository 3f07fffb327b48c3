/*
 * gao.h -- CPU oracle for the genetic algorithm that searches for Hadamard
 * matrices (Balogh & Ruiz, "A GPU accelerated Genetic Algorithm for the
 * Construction of Hadamard Matrices", arXiv 2208.14961).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the GPU library is checked against.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no source with the GPU library.
 *
 * Data layout (paper, Sec. 3.4): a population of n matrices of order m is an
 * int8 array pop[n][m][m]; entry (row i, column j) of matrix k is
 * pop[k*m*m + i*m + j] and holds +1 or -1.
 *
 * Every random choice is a pure function of (seed, stream, generation,
 * index, draw) through Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11), implemented here from that
 * paper.
 *
 * Parity status per function (pins live in tests/):
 *   gao_philox4x32_10    pinned: published known-answer vectors.
 *   gao_gram, gao_fitness pinned: Sylvester and Paley matrices (fitness 0),
 *                         the exhaustive m=4 census, closed forms for the
 *                         all-equal-columns matrix, the row-space identity.
 *   gao_init_population  pinned: invariants, exact pattern counts at m=4,
 *                         chi-square uniformity of column patterns.
 *   gao_crossover        pinned: the paper's crossover figure, exhaustive
 *                         m=4 column-origin check.
 *   gao_mutate           pinned: the paper's mutation figure, panels (b),
 *                         (c), (d) as printed, panel (a) with its index pairs
 *                         read from the figure's colours.
 *   gao_step, gao_run    pinned by composition of the above, by invariants,
 *                         and by selection-distribution tests; the exact
 *                         bytes of a whole run are "parity unpinned" beyond
 *                         agreement with the independent GPU implementation.
 *   gao_draw stream/counter mapping: a convention of this project, "parity
 *                         unpinned" except through the Philox vectors.
 */
#ifndef GAO_H
#define GAO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* fitness kinds: the key each individual is ranked by (smaller is fitter) */
enum {
  GAO_FIT_SQ = 0,          /* sum over column pairs i<j of (c_i . c_j)^2     */
  GAO_FIT_ABS = 1,         /* sum over i<j of |c_i . c_j|   (= F1 / 2)       */
  GAO_FIT_NNZ = 2,         /* number of i<j with c_i . c_j != 0 (= F2 / 2)  */
  GAO_FIT_SQ_PLUS_NNZ = 3, /* SQ + NNZ                                       */
  GAO_FIT_F1 = 4,          /* paper Eq. (fitness0): sum |Q^T Q| - m^2        */
  GAO_FIT_F2 = 5           /* paper Eq. (fitness):  nnz(Q^T Q) - m           */
};

enum { GAO_SEL_TOURNAMENT = 0, GAO_SEL_PAPER = 1 };

/* largest order: Table 2 of the paper times orders up to 100 */
enum { GAO_MAX_M = 128 };

/* Philox stream tags: partition the draw namespace by purpose */
enum {
  GAO_STREAM_INIT = 1,
  GAO_STREAM_SELECT = 2,
  GAO_STREAM_XOVER = 3,
  GAO_STREAM_MUTATE = 4,
  GAO_STREAM_PERM = 5
};

typedef struct {
  uint32_t m;               /* order, multiple of 4, 4..GAO_MAX_M           */
  uint32_t n;               /* population size                              */
  uint64_t seed;            /* Philox key                                   */
  uint32_t fitness;         /* GAO_FIT_*                                    */
  uint32_t selection;       /* GAO_SEL_*                                    */
  uint32_t tournament_k;    /* contestants per tournament, >= 1             */
  uint32_t elite;           /* elites kept per generation (tournament mode) */
  uint64_t xo_threshold;    /* crossover iff draw < threshold; 2^32 = always */
  uint64_t mut_threshold;   /* mutation iff draw < threshold; 2^32 = always  */
  uint32_t nc;              /* mutated columns per mutated child            */
  uint32_t nr;              /* row pairs per mutated child                  */
  uint32_t max_generations; /* generation budget                            */
  uint32_t stop_on_found;   /* stop as soon as some key is 0                */
  uint32_t mut_shared;      /* 1: the first mutation method of Sec. 3.5:
                               every mutated child of a generation takes
                               the same columns and row pairs, drawn once
                               per generation (index GAO_SHARED_MUTATION) */
} gao_config;

/* the draw index of the per-generation mutation of mut_shared (above every
 * child index) */
#define GAO_SHARED_MUTATION 0xFFFFFFFFu

typedef struct {
  int32_t found;        /* 1 if a key of 0 was reached                     */
  uint32_t generation;  /* generation holding the reported individual     */
  uint32_t index;       /* slot of the best individual (lowest on ties)   */
  uint32_t best_key;    /* its key                                         */
} gao_result;

/* 0 on success, -1 on an invalid configuration */
int gao_validate(const gao_config* cfg);

void gao_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);
uint32_t gao_draw(uint64_t seed, uint32_t stream, uint32_t gen, uint32_t idx,
                  uint32_t d);
uint32_t gao_bounded(uint32_t u, uint32_t range);

void gao_gram(uint32_t m, const int8_t* Q, int32_t* G);
/* comps (nullable): SQ, ABS, NNZ of one matrix; returns the key */
uint32_t gao_fitness_one(uint32_t m, uint32_t kind, const int8_t* Q,
                         uint32_t* comps);
int gao_fitness(const gao_config* cfg, const int8_t* pop, uint32_t* keys,
                uint32_t* comps);

int gao_init_population(const gao_config* cfg, int8_t* pop);

void gao_crossover(uint32_t m, const int8_t* A, const int8_t* B, uint32_t cut,
                   int8_t* O0, int8_t* O1);
/* cols[nc], r1[nr], r2[nr]; applies the flips in column-major order */
void gao_mutate(uint32_t m, int8_t* Q, uint32_t nc, const uint32_t* cols,
                uint32_t nr, const uint32_t* r1, const uint32_t* r2);

uint32_t gao_permute(uint64_t seed, uint32_t gen, uint32_t domain, uint32_t s);
/* sel_out[count]: the count smallest (key, index), listed by index */
void gao_select_set(const uint32_t* keys, uint32_t n, uint32_t count,
                    uint32_t* sel_out);
/* parents of child pair p when producing generation gen_out (tournament) */
void gao_tournament_parents(const gao_config* cfg, const uint32_t* keys,
                            uint32_t gen_out, uint32_t p, uint32_t* a,
                            uint32_t* b);

int gao_step(const gao_config* cfg, const int8_t* pop_in,
             const uint32_t* keys_in, int8_t* pop_out, uint32_t* keys_out,
             uint32_t gen_in);
/* runs from gen 0; on return pop_final holds the last generation */
int gao_run(const gao_config* cfg, int8_t* pop_final, uint32_t* keys_final,
            gao_result* res);

/* count of matrices violating: column 0 all +1, other columns balanced */
uint32_t gao_check_invariants(uint32_t m, uint32_t n, const int8_t* pop);

int gao_num_threads(void);
/* Threads of the OpenMP loops from now on (results do not depend on it). */
void gao_set_num_threads(int threads);

#ifdef __cplusplus
}
#endif
#endif
