/*
 * ga.h -- C ABI of libga, the MI355X (gfx950) implementation of the
 * per-generation hot path of the genetic algorithm for Hadamard matrices of
 * Balogh & Ruiz ("A GPU accelerated Genetic Algorithm for the Construction
 * of Hadamard Matrices", arXiv 2208.14961).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Population layout ("packed").  A population of n matrices of order m is an
 * array of uint32 words pop[n][m][W], W = 1 for m <= 32, 2 for m <= 64 and
 * 4 for m <= 128 (above order 64 a column is one 16-byte group; its words
 * past ceil(m / 32) are 0).  Column j of matrix k occupies words
 * pop[k][j][0..W-1]; bit (r % 32) of word r / 32 is 1 iff entry (row r,
 * column j) is -1.  Bits for rows >= m are 0.  The paper
 * stores int8 entries Q[m*m*k + m*i + j] (Sec. 3.4); this layout holds the
 * same matrices with one bit per entry, so that the dot product of two
 * columns is c_i . c_j = m - 2 * popcount(x_i xor x_j).
 *
 * Invariants (Sec. 3.1).  Column 0 of every matrix is all +1 (its words are
 * 0) and every other column is balanced (m/2 entries -1).  Initialization,
 * crossover (whole columns, Sec. 3.4) and mutation (flips of unequal entry
 * pairs only, Sec. 3.5) keep them.  The fitness kernels rely on them: pairs
 * involving column 0 are orthogonal and are skipped.
 *
 * Keys.  Each individual's fitness key is a uint32, smaller is fitter, and 0
 * exactly for Hadamard matrices.  With G = Q^T Q and pairs i < j of columns:
 *   GA_FIT_SQ            sum G_ij^2
 *   GA_FIT_ABS           sum |G_ij|              (= F1 / 2)
 *   GA_FIT_NNZ           #{G_ij != 0}            (= F2 / 2)
 *   GA_FIT_SQ_PLUS_NNZ   SQ + NNZ
 *   GA_FIT_F1            sum_{i,j} |G_ij| - m^2  (Sec. 3.2, Eq. fitness0)
 *   GA_FIT_F2            nnz(G) - m              (Sec. 3.2, Eq. fitness)
 * Components (optional) are the triple (SQ, ABS, NNZ) per individual.
 *
 * Randomness.  Every random choice is word d % 4 of the Philox4x32-10 block
 * (Salmon et al., SC'11) with counter (d / 4, index, generation, stream) and
 * key (seed low 32 bits, seed high 32 bits).  Streams: 1 initialization,
 * 2 selection, 3 crossover (and the per-child mutation coin), 4 mutation,
 * 5 parent permutation.  Bounded integers are floor(u * range / 2^32);
 * a coin with threshold t (0 <= t <= 2^32) succeeds iff u < t.
 *
 * Device pointers and streams.  Unless stated otherwise, pointer arguments
 * are device pointers owned by the caller, and `stream` is a hipStream_t
 * (NULL = the null stream).  Calls marked "async" only enqueue work.
 *
 * Errors.  No call aborts or throws.  Each returns a ga_status; on error
 * ga_last_error() gives a message for the calling thread.
 */
#ifndef GA_H
#define GA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GA_OK = 0,
  GA_PENDING = 1,     /* ga_poll: the request has not finished yet          */
  GA_EINVAL = -1,     /* invalid configuration or argument                   */
  GA_ENOMEM = -2,     /* device allocation failed                            */
  GA_EDEVICE = -3,    /* a HIP call failed; see ga_last_error()              */
  GA_EBUDGET = -4,    /* a request can never fit the server's HBM budget     */
  GA_ENOTFOUND = -5,  /* unknown request id                                  */
  GA_ESTOPPED = -6    /* the server has stopped (ga_server_stop)             */
} ga_status;

typedef enum {
  GA_FIT_SQ = 0,
  GA_FIT_ABS = 1,
  GA_FIT_NNZ = 2,
  GA_FIT_SQ_PLUS_NNZ = 3,
  GA_FIT_F1 = 4,
  GA_FIT_F2 = 5
} ga_fitness_kind;

typedef enum {
  /* Tournament selection over the previous generation, optional elitism.  */
  GA_SEL_TOURNAMENT = 0,
  /* The paper's truncation (Sec. 3.3): n = 4N; the best 2N of the 4N
   * matrices become the parents in random order; pairs (P_k, P_{k+N}) make
   * offspring O_k, O_{N+k} in slots 2N + k and 3N + k.                      */
  GA_SEL_PAPER = 1
} ga_selection_kind;

enum {
  GA_STOP_ON_FOUND = 1u, /* ga_run: stop at the first generation with key 0 */
  /* The first mutation method of Sec. 3.5: every mutated child of a
   * generation takes the same nc columns and nr row pairs, the draws of
   * index 0xFFFFFFFF (above every child index) in stream 4; without it each
   * child q draws its own (index q, the third method).                     */
  GA_MUT_SHARED = 2u,
  /* Lanes per child in the children kernel (the tile shape), bits 8..12 of
   * flags: 0 lets the library choose (ga_run of at least 193 generations
   * times the candidates on its own first generations, launched one by one,
   * and remembers the choice per run shape; otherwise the tuning table);
   * 2, 4, 8 or 16 force it (orders 36..64: 4 or 8; orders 68..128: 8 or
   * 16).  Results do not depend on it.                                     */
  GA_LANES_SHIFT = 8u,
  GA_LANES_MASK = 0x1F00u,
  /* How ga_fitness and ga_fitness_repeat form the Gram products (Sec. 3.2),
   * bits 13..14 of flags: 0 lets the library's table choose per order,
   * GA_GRAM_PACKED forces xor + popcount on the packed columns, GA_GRAM_MFMA
   * the int8 matrix-core path (orders 36..128 only: G_ij = 4 s_ij - m with
   * s = X^T X over the 0/1 indicator X of the -1 entries).  Results do not
   * depend on it.                                                          */
  GA_GRAM_SHIFT = 13u,
  GA_GRAM_MASK = 0x6000u,
  GA_GRAM_PACKED = 1u << 13,
  GA_GRAM_MFMA = 2u << 13
};

enum { GA_MAX_M = 128 };  /* largest order */

typedef struct {
  uint32_t m;               /* order: m % 4 == 0, 4 <= m <= GA_MAX_M         */
  uint32_t n;               /* population size (>= 2; paper mode: n = 4N)    */
  uint64_t seed;            /* Philox key                                    */
  uint32_t fitness;         /* ga_fitness_kind                               */
  uint32_t selection;       /* ga_selection_kind                             */
  uint32_t tournament_k;    /* contestants per tournament, 1..64             */
  uint32_t elite;           /* tournament mode: elites kept, < n, <= 65536;
                               paper mode: must be 0                         */
  uint64_t xo_threshold;    /* crossover coin threshold, <= 2^32             */
  uint64_t mut_threshold;   /* per-child mutation coin threshold, <= 2^32    */
  uint32_t nc;              /* mutated columns per mutated child, <= 64      */
  uint32_t nr;              /* row pairs per mutated child, <= 64            */
  uint32_t max_generations; /* generation budget of ga_run, < 2^31          */
  uint32_t flags;           /* GA_STOP_ON_FOUND | GA_MUT_SHARED |
                               lanes << GA_LANES_SHIFT | GA_GRAM_*           */
} ga_config;

typedef struct {
  int32_t found;        /* 1 iff best_key == 0                               */
  uint32_t generation;  /* generation of the reported population             */
  uint32_t index;       /* slot of its best individual (lowest on ties)      */
  uint32_t best_key;    /* that individual's key                             */
  int8_t matrix[GA_MAX_M * GA_MAX_M]; /* that individual, int8 +1/-1,
                                         row-major m x m                     */
} ga_result;

/* Message describing the calling thread's last error ("" if none). */
const char* ga_last_error(void);

/* GA_OK iff the configuration is valid (limits as documented above). */
ga_status ga_validate(const ga_config* cfg);

/* Number of uint32 words of one packed population: n * m * W (W as in the
 * layout above); 0 for an invalid order. */
size_t ga_population_words(const ga_config* cfg);

/*
 * Initial population (Sec. 3.1).  Async.  pop: [n][m][W] words, written.
 * Column 0 is all +1; column j >= 1 starts with rows 0..m/2-1 equal to -1
 * and the rest +1, then is shuffled by Fisher-Yates: for i1 = 0..m-2,
 * i2 = i1 + bounded(draw(stream 1, generation 0, index k, d = j*m + i1),
 * m - i1), swap rows i1 and i2.
 */
ga_status ga_init_population(const ga_config* cfg, uint32_t* pop,
                             void* stream);

/*
 * Fitness of every individual (Sec. 3.2, Sec. 4.2).  Async.
 * pop: [n][m][W] words, read.  keys: [n] written with cfg->fitness's key.
 * comps: nullable; [n][3] written with (SQ, ABS, NNZ).
 */
ga_status ga_fitness(const ga_config* cfg, const uint32_t* pop,
                     uint32_t* keys, uint32_t* comps, void* stream);

/*
 * Lanes per child that ga_run would use now for this configuration (the
 * children kernel's tile shape): the forced value, else the one measured by
 * an earlier run of the same shape in this process, else the tuning
 * table's.  0 if the configuration is invalid.  Host only.
 */
uint32_t ga_tuned_lanes(const ga_config* cfg);

/*
 * The same Gram + fitness (Sec. 3.2), evaluated `reps` times over the whole
 * population inside one launch: a throughput form of ga_fitness for
 * measuring the Gram + fitness core without per-launch overhead.  Async.
 * pop: [n][m][W] words, read.  keys: [n], written with cfg->fitness's key
 * (every evaluation writes the same value; the result equals ga_fitness's).
 * reps >= 1 and n * reps < 2^40, else GA_EINVAL.
 */
ga_status ga_fitness_repeat(const ga_config* cfg, const uint32_t* pop,
                            uint32_t* keys, uint32_t reps, void* stream);

/*
 * One generation, gen_in -> gen_in + 1 (Sec. 3, the loop body).  Async.
 * pop_in/keys_in (read) hold generation gen_in with its keys; pop_out and
 * keys_out (written, must not overlap the inputs) receive generation
 * gen_in + 1 and its keys.  With G = gen_in + 1:
 *
 * Tournament mode.  e = cfg->elite.  Slots 0..e-1 receive the e individuals
 * with the smallest (key, index), in increasing index order, unchanged.
 * Child pair p = 0..ceil((n-e)/2)-1 has parents a, b: parent s in {0, 1} is
 * the contestant with the smallest (key, index) among x_c = bounded(
 * draw(2, G, p, s*t + c), n), c < t.  With u = draw(3, G, p, .): if
 * u_0 < xo_threshold, cut = 1 + bounded(u_1, m - 1), child 0 takes columns
 * < cut from a and the rest from b, child 1 the complement (Sec. 3.4);
 * otherwise the children copy a and b.  Child c of the pair goes to slot
 * e + 2p + c (dropped if >= n).  It is mutated iff u_{2+c} < mut_threshold:
 * with q = 2p + c, columns col_jc = 1 + bounded(draw(4, G, q, jc), m - 1),
 * jc < nc, row pairs r1 = bounded(draw(4, G, q, nc + 2 ir), m),
 * r2 = bounded(draw(4, G, q, nc + 2 ir + 1), m), ir < nr; for each jc in
 * order, for each ir in order, the entries (r1, col) and (r2, col) are
 * negated iff they differ (Sec. 3.5, third method).  With GA_MUT_SHARED,
 * q = 0xFFFFFFFF for every child: one set of columns and row pairs per
 * generation (Sec. 3.5, first method, for nc = nr = 1).
 *
 * Paper mode (Sec. 3.3-3.5).  N = n / 4.  The 2N individuals with the
 * smallest (key, index), listed in index order as sel[0..2N-1], move to
 * parent slots s = 0..2N-1 as sel[pi(s)] (keys carried along), where pi is a
 * keyed permutation of [0, 2N): an eight-round Feistel network on 2h bits
 * (4^h >= 2N), round r mapping (L, R) to (R, L xor (draw(5, G, R, r) mod
 * 2^h)), cycle-walked into [0, 2N).  Pair k < N makes its children from
 * parent slots k and k + N exactly as above and writes them to slots
 * 2N + k and 3N + k.
 *
 * Elitism and paper mode rank keys below 2^24.  Every kind fits up to
 * order 76; from order 80 on, the SQ and SQ + NNZ keys of some matrices do
 * not (the largest SQ key is C(m-1, 2) * m^2), so ga_validate rejects those
 * kinds with elitism or paper mode there.  Tournaments without elites
 * compare whole keys and take every kind at every order.
 */
ga_status ga_step(const ga_config* cfg, const uint32_t* pop_in,
                  const uint32_t* keys_in, uint32_t* pop_out,
                  uint32_t* keys_out, uint32_t gen_in, void* stream);

/*
 * ga_step without device allocation, for callers that cannot allocate
 * (work under HIP graph capture, serving loops that forbid allocation).
 * Same arguments, validation and results as ga_step.  Its run state and
 * selection workspace live in a fixed device array of the library
 * (288.5 KiB per device, held until the process ends) that covers every
 * population the library accepts (n <= 2^24; larger n is GA_EINVAL); the
 * call clears what must start at zero with a kernel of its own, so it
 * enqueues no memset and no allocation, and can be captured.  Every call on
 * one device shares that array: calls that overlap on one device (two
 * streams, or two threads) race and must be ordered by the caller.  Async.
 */
ga_status ga_step_static(const ga_config* cfg, const uint32_t* pop_in,
                         const uint32_t* keys_in, uint32_t* pop_out,
                         uint32_t* keys_out, uint32_t gen_in, void* stream);

/*
 * The truncation selection of paper mode (Sec. 3.3) as ga_run makes it for
 * populations up to 65,536: of the n keys of one generation, the n/2
 * smallest (key, index) pairs, listed in index order.  cfg: a valid
 * paper-mode config with n <= 65536 (else GA_EINVAL).  Buffers are device
 * memory owned by the caller:
 *   keys: n keys, none above the largest key of cfg's fitness kind at its
 *     order (the search with no threshold known starts there).
 *   threshold: one word.  In: a key value with at least n/2 keys at or below
 *     it (in a run, the previous generation's threshold: it never rises), or
 *     0xFFFFFFFF when none is known; the counts start in a window of 1024
 *     values below it.  Out: the threshold T, the (n/2)-th smallest key.
 *   sel: n/2 words: the selected indices in increasing order (every key
 *     below T and, in index order, the first keys equal to T that make n/2).
 * ga_run's paper mode writes the same ranks through the generation's parent
 * permutation instead.  Two launches over tiles of 4096 keys, on the
 * stream's workspace (calls on one stream are ordered).  Async.
 */
ga_status ga_paper_select(const ga_config* cfg, const uint32_t* keys, uint32_t* threshold,
                          uint32_t* sel, void* stream);

/*
 * A whole run (Sec. 3, the algorithm; Sec. 6 loop): init, fitness, then
 * ga_step until a generation holds a key of 0 (with GA_STOP_ON_FOUND) or
 * max_generations steps were made.  Synchronous: returns when done.
 * pop_a, pop_b: two population buffers; generation g is left in pop_a if g
 * is even, pop_b if odd.  keys_a, keys_b likewise.  out (host pointer) gets
 * the final generation, its best (key, index) and that matrix.
 */
ga_status ga_run(const ga_config* cfg, uint32_t* pop_a, uint32_t* pop_b,
                 uint32_t* keys_a, uint32_t* keys_b, ga_result* out,
                 void* stream);

/*
 * Several independent runs advanced together: one children launch per order
 * and generation covers every active run of that order.  Selection is shared
 * the same way: the order's elitist runs choose their elites in one launch,
 * its paper-mode runs (up to 65,536 individuals) select in one pair of
 * launches; larger paper-mode runs add launches of their own.  Each run's
 * selection works in its own allocation.  Synchronous.  cfgs, outs: host arrays of count entries.  The library
 * allocates the populations.  Every run's result equals what ga_run gives
 * for it alone.
 */
ga_status ga_run_batch(const ga_config* cfgs, uint32_t count, ga_result* outs,
                       void* stream);

/*
 * Layout conversion between the paper's int8 matrices (Sec. 3.4: entry (row
 * i, column j) of matrix k at q[k*m*m + i*m + j], values +1 and -1) and the
 * packed layout above.  Async; one pass over each array.
 * ga_pack: q [n][m][m] int8 (read), pop [n][m][W] (written): an entry packs
 * as -1 iff it is negative.  bad: NULL, or a device uint32 that is
 * increased by the number of entries other than +1 and -1.
 * ga_unpack: pop (read), q (written) with +1 and -1.
 * Neither checks the invariants (ga_check_invariants does).
 */
ga_status ga_pack(const ga_config* cfg, const int8_t* q, uint32_t* pop,
                  uint32_t* bad, void* stream);
ga_status ga_unpack(const ga_config* cfg, const uint32_t* pop, int8_t* q,
                    void* stream);

/* Count (on the host, synchronously) the matrices of pop breaking the
 * invariants: column 0 words not 0, a column not balanced, bits set above
 * row m - 1. */
ga_status ga_check_invariants(const ga_config* cfg, const uint32_t* pop,
                              uint32_t* bad_count, void* stream);

/*
 * Timing, for measurement.  While enabled, ga_run records HIP events on its
 * stream around its generation loop (the chunks of children launches, one
 * launch per generation; not the generations a lanes measurement makes one
 * by one before the chunks).  ga_timing_read returns the mean time per
 * generation in milliseconds and the number of generations timed since the
 * last ga_timing_enable(1).  Not thread-safe; meant for benchmarks.
 */
ga_status ga_timing_enable(int on);
ga_status ga_timing_read(double* mean_ms, uint64_t* launches);

/* -------------------------------------------------------------------------
 * Search server: continuous batching of independent runs (every selection
 * mode, as ga_run_batch).
 * Requests are admitted in arrival order among those whose device memory
 * fits the HBM budget (one that does not fit is passed over by at most 64
 * later admissions, then waited for);
 * admitted populations stay resident on the device and advance one
 * generation per server tick together with every other active request; a
 * request retires when a key reaches 0 (with GA_STOP_ON_FOUND) or its
 * budget is spent.  Each result equals ga_run's for the same config.
 * ---------------------------------------------------------------------- */
typedef struct ga_server ga_server;

/* Starts the server's worker thread on `device`.  *out: new handle. */
ga_status ga_server_create(uint64_t hbm_budget_bytes, int device,
                           ga_server** out);
/* Non-blocking.  GA_EBUDGET if the request alone exceeds the budget.  Once
 * the worker has stopped, every submission is refused with its terminal
 * status: GA_ESTOPPED after ga_server_stop, the device error's status
 * (GA_EDEVICE, GA_ENOMEM) if one ended it. */
ga_status ga_submit(ga_server* srv, const ga_config* cfg, uint64_t* request_id);
/* GA_PENDING while running, GA_OK once *out holds the result. */
ga_status ga_poll(ga_server* srv, uint64_t request_id, ga_result* out);
/* Blocks until the request finishes; then as ga_poll. */
ga_status ga_wait(ga_server* srv, uint64_t request_id, ga_result* out);
/* Seconds from submission to retirement of a finished request. */
ga_status ga_request_latency(ga_server* srv, uint64_t request_id,
                             double* seconds);
/* Stops the worker: requests not yet finished fail with GA_ESTOPPED (a
 * device error ends the worker the same way, with its own status); finished
 * results stay readable with ga_poll / ga_wait until ga_server_destroy.
 * Blocks until the worker has exited. */
ga_status ga_server_stop(ga_server* srv);
/* Stops the worker as ga_server_stop does and frees the server. */
ga_status ga_server_destroy(ga_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* GA_H */
