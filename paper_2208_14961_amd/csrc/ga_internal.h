// ga_internal.h -- structures and launchers shared by libga's own sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ga.h"

namespace ga {

// Words per packed column: 1 up to order 32, 2 up to 64, 4 up to 128 (a
// column of a larger order is one 16-byte group; its unused words are 0).
__host__ __device__ constexpr uint32_t col_words(uint32_t m) {
  return m <= 32 ? 1u : (m <= 64 ? 2u : 4u);
}

// The largest key of a fitness kind at order m (all columns equal: every
// pair has |c_i . c_j| = m).
__host__ __device__ inline uint64_t max_key(uint32_t m, uint32_t kind) {
  const uint64_t P = (uint64_t)(m - 1) * (m - 2) / 2, mm = m;
  switch (kind) {
    case GA_FIT_SQ: return P * mm * mm;
    case GA_FIT_ABS: return P * mm;
    case GA_FIT_NNZ: return P;
    case GA_FIT_SQ_PLUS_NNZ: return P * mm * mm + P;
    case GA_FIT_F1: return 2 * P * mm;
    default: return 2 * P;
  }
}

constexpr uint32_t kMaxN = 1u << 24;        // population size limit
constexpr uint32_t kMaxElite = 1u << 16;    // elite count limit
// generation budget limit: generation numbers up to the budget plus two
// chunks of launches stay below 2^32
constexpr uint32_t kMaxGenerations = 0x7fffffffu;
constexpr uint32_t kKeyBits = 24;           // selection ranks keys < 2^24
constexpr int kBlock = 256;                 // threads per block, bulk kernels
constexpr int kChildBlock = 64;             // one wave per block: children
constexpr int kQuadChildren = 16;           // children per block, orders <= 32
constexpr int kOctChildren = 8;             // children per block, orders >= 36
constexpr int kOrders = GA_MAX_M / 4;       // orders 4, 8, .., 128
constexpr int kSelTile = 512;               // elements per block, selection
constexpr uint64_t kMaxPermTable = 1u << 24;  // entries of a chunk's slot table
constexpr uint32_t kBatchTableRows = 32;      // generations per batched chunk with a table
constexpr int kMaxSelBlocks = kMaxN / kSelTile;

// Device-resident progress of one run.  Generation g of the run lives in
// buffer A if g is even, B if odd.  Launches are issued in chunks: launch i
// of a chunk (its "node") produces generation G = gen_base + i + 1, and a
// small kernel after the chunk advances gen_base.  A generation runs only if
// G <= max_gen and, when stopping on a solution, no earlier generation held
// a key of 0.  No per-block fences or counters are needed: each kernel
// boundary orders the generations.
struct RunState {
  unsigned long long best;  // (key << 32 | slot) of the reported generation
  uint32_t gen_base;        // generations completed before the current chunk
  uint32_t found_gen;       // first generation holding a key of 0, or ~0u
  uint32_t final_gen;       // reported generation (set by the finish kernel)
  uint32_t pad[3];
};

// Host-side view: has the run finished after the chunks launched so far?
inline bool run_done(const RunState& s, uint32_t max_gen, bool stop_on_found) {
  return s.gen_base >= max_gen || (stop_on_found && s.found_gen <= s.gen_base);
}

// One population in a step launch.
struct SelWork;

// Elitism inside ga_run.  Generation G's elites are the e smallest (key,
// slot) of generation G - 1, in slots 0 .. e-1 of G, so they precede every
// child on ties: the e smallest of G are among those elites and the
// children whose key is below kstar, the largest elite key.  The children
// launch of G copies the elites (src) and appends such children to short
// candidate lists; one single-block launch then picks the next elites from
// the elites and those lists.
struct EliteWork {
  uint32_t kstar;            // largest key among the elites of the generation
                             // the next children launch makes
  uint32_t pad[63];
  uint32_t src[kMaxElite];   // elite s of that generation is row src[s] of
                             // the one before (increasing)
};

// Paper mode in ga_run up to kPaperTileMaxN individuals (ga_paper.hip): a
// launch over tiles of kPaperTile keys counts each tile's keys in a window of
// kPaperBins values below the previous threshold; a second launch over the
// tiles finds the threshold in every tile and lists the selected indices in
// index order.
constexpr uint32_t kPaperTile = 4096;
constexpr uint32_t kPaperBins = 1024;
constexpr uint32_t kPaperTileMaxN = 65536;
constexpr uint32_t kPaperMaxTiles = kPaperTileMaxN / kPaperTile;
struct PaperWork {
  uint32_t T[2];    // threshold of the selection of generation g's parents in
                    // T[g & 1]; ~0 before the first
  uint32_t pad[62];
  uint32_t hist[kPaperMaxTiles][kPaperBins + 1];  // per tile, entry d: its keys with
                                                  // d <= top - key < kPaperBins;
                                                  // last: its keys below that window
};

// The candidate lists of an elitist run: a child below the largest elite key
// is appended, as (slot, key), to list (its block's index in the population)
// mod kEliteLists with one atomic per block.  A block holds at most 32
// children, so a list receives at most ceil(n / kEliteLists) + 33 entries.
// The area holds the lists' counts, their entries (list j from entry
// j * elite_list_cap(n)), then the selection's scratch for lists too long
// for its LDS: a bitmap and a prefix count per 32 slots, the items' keys
// and their slots (n each).
constexpr uint32_t kEliteLists = 256;
__host__ __device__ inline uint32_t elite_list_cap(uint32_t n) {
  return (n + kEliteLists - 1) / kEliteLists + 33;
}
inline size_t elite_area_words(uint32_t n) {
  const size_t nw = ((size_t)n + 31) / 32;
  return kEliteLists + (size_t)kEliteLists * elite_list_cap(n) * 2 + 2 * nw + 2 * (size_t)n;
}

struct PopDesc {
  uint32_t* pop_a;
  uint32_t* pop_b;
  uint32_t* keys_a;
  uint32_t* keys_b;
  RunState* state;
  uint64_t seed;
  uint64_t xo_thr;
  uint64_t mut_thr;
  uint32_t m, n;
  uint32_t elite;        // first child slot (tournament); 2N (paper)
  uint32_t nchild;       // children produced per generation
  uint32_t t, nc, nr, kind;
  uint32_t paper;        // 1: paper mode (parents in slots k, k+N of output)
  uint32_t max_gen;
  uint32_t stop_on_found;
  uint32_t block_begin;  // first block of this population in the launch
  uint32_t nblocks;      // blocks of this population
  uint32_t lanes;        // lanes per child in the children kernel
  uint32_t lanes_forced; // 1: lanes come from the config, not the table
  uint32_t mut_shared;   // 1: one mutation draw set per generation (Sec. 3.5, first method)
  SelWork* sel;          // batched and served runs with elitism or paper mode: their
                         // selection workspace (null otherwise)
  uint32_t* slots;       // batched and served paper-mode runs: kBatchTableRows rows of
                         // slot permutations for a chunk (null: walked inline)
  EliteWork* ew;         // ga_run with elitism: the children launch copies the elites
                         // and appends candidates (null: elites copied by the selection)
  uint32_t* ecount;      // with ew: the kEliteLists candidate counts (see elite_list_cap)
  uint2* elist;          // with ew: the candidate lists, list j from entry j * ecap
  uint32_t* escratch;    // with ew: the selection's scratch for long lists
  uint32_t ecap;         // with ew: entries per candidate list
  PaperWork* pw;          // ga_run paper mode up to kPaperTileMaxN: the tile
                         // selection's work area
  uint32_t* psel;        // with pw: the selected indices of generation G - 1 in
                         // index order (2N); parent slot s of G receives
                         // psel[pfwd[s]]
  const uint32_t* pfwd;  // with pw: the chunk's forward slot table, rows of 2N
};

// Workspace of the selection pipeline of one population.
struct SelWork {
  uint32_t h1[4096];
  uint32_t h2[4096];
  uint32_t blk_less[kMaxSelBlocks];
  uint32_t blk_eq[kMaxSelBlocks];
  uint32_t bucket, below, T, r;   // results of the radix select
};

// ---- the Gram products of the standalone fitness ---------------------------
constexpr uint32_t kMfmaMinOrder = 36;  // the int8 MFMA path: orders 36..128
// Whether ga_fitness / ga_fitness_repeat use the MFMA path for c: forced by
// its flags, else the measured choice per order (ga_tuning.hip).
bool use_mfma(const ga_config* c);
// Gram + fitness on the matrix cores (ga_mfma.hip): evaluation e < total is
// individual e mod n; comps and st as in launch_fitness (st only when total
// is n); a grid sized for `cus` compute units.
hipError_t launch_fitness_mfma(const ga_config* c, const uint32_t* pop, uint32_t* keys,
                               uint32_t* comps, RunState* st, uint64_t total, uint32_t cus,
                               hipStream_t s);

// ---- launchers (ga_kernels.hip, ga_children.hip, ga_select.hip) ---------
hipError_t launch_init(const ga_config* c, uint32_t* pop, hipStream_t s);
// keys for all n; comps nullable; st nullable, else a key of 0 in generation
// 0 sets st->found_gen = 0
hipError_t launch_fitness(const ga_config* c, const uint32_t* pop,
                          uint32_t* keys, uint32_t* comps, RunState* st,
                          hipStream_t s);
// keys of all n, the population evaluated reps times in one launch over a
// grid sized for `cus` compute units
hipError_t launch_fitness_repeat(const ga_config* c, const uint32_t* pop,
                                 uint32_t* keys, uint32_t reps, uint32_t cus,
                                 hipStream_t s);
// selection of the `count` smallest (key, index) of generation G - 1 into
// generation G (elitism: slot = rank in index order; paper mode: slot =
// pi^-1(rank)), G from the state and the launch's node.  slots: paper mode's
// pi^-1 for this launch's generation from launch_perm_table, or null to
// evaluate it inline.
// src_out, kstar_out (elitism in ga_run): write the sources of the selected
// ranks and the threshold key there instead of copying the rows.
hipError_t launch_select(const PopDesc& d, uint32_t count, SelWork* ws,
                         uint32_t node, const uint32_t* slots, hipStream_t s,
                         uint32_t* src_out = nullptr, uint32_t* kstar_out = nullptr);
// paper mode: pi^-1 over [0, count) for the generations of launches
// 0 .. nodes-1 of a chunk, row by row into out[nodes][count]; forward: pi
hipError_t launch_perm_table(const PopDesc& d, uint32_t count, uint32_t nodes,
                             uint32_t* out, hipStream_t s, bool forward = false);
// ga_run with elitism: the elites of generation gen_base + node + 1 of d
// chosen from generation gen_base + node (see EliteWork), from its elites
// and its listed children.  (The first generation's come from launch_select
// with src_out.)
hipError_t launch_elite_select(const PopDesc& d, uint32_t node, hipStream_t s);
// Points d's candidate lists and scratch into an area of
// elite_area_words(d->n) words.
inline void set_elite_area(PopDesc* d, uint32_t* area) {
  d->ecap = elite_list_cap(d->n);
  d->ecount = area;
  d->elist = reinterpret_cast<uint2*>(area + kEliteLists);
  d->escratch = area + kEliteLists + (size_t)kEliteLists * d->ecap * 2;
}
// The same for several runs in one launch (block b: run descs[runs[b]]).
hipError_t launch_elite_select_multi(const PopDesc* descs_dev, const uint32_t* runs,
                                     uint32_t count, uint32_t node, hipStream_t s);
// Paper mode up to kPaperTileMaxN, parents of generation gen_base + node + 1
// (d.pw holds the previous threshold, or ~0): the threshold and the tile
// offsets, then sel[rho] = the rho-th selected index in index order.
hipError_t launch_paper_select(const PopDesc& d, uint32_t node, uint32_t* sel, hipStream_t s);
// The same for several runs in two launches: block b takes tile (e & 15) of
// run descs[e >> 4], e = tiles[b], into that run's d.psel.
hipError_t launch_paper_select_multi(const PopDesc* descs_dev, const uint32_t* tiles,
                                     uint32_t nblocks, uint32_t node, hipStream_t s);
// children of every population in descs (device array), all of order m
hipError_t launch_children(const PopDesc* descs_dev, const uint32_t* block_pop,
                           uint32_t total_blocks, uint32_t m, uint32_t lanes,
                           uint32_t node, hipStream_t s);
// children of one population (descriptor passed by value)
hipError_t launch_children_one(const PopDesc& d, uint32_t node, hipStream_t s);
// gen_base += k for every population of the table
hipError_t launch_advance(const PopDesc* descs_dev, uint32_t ndesc, uint32_t k,
                          hipStream_t s);
hipError_t launch_advance_one(RunState* st, uint32_t k, hipStream_t s);
// final generation of every population of the table and its best (key, slot)
hipError_t launch_finish(const PopDesc* descs_dev, uint32_t ndesc,
                         hipStream_t s);
hipError_t launch_finish_one(const PopDesc& d, hipStream_t s);
hipError_t launch_reset_state(RunState* st, hipStream_t s);
// state for a single step from generation gen (no stop condition)
hipError_t launch_set_state(RunState* st, uint32_t gen, hipStream_t s);
hipError_t launch_check(const ga_config* c, const uint32_t* pop,
                        uint32_t* bad, hipStream_t s);
// int8 [n][m][m] <-> packed; bad nullable
hipError_t launch_pack(const ga_config* c, const int8_t* q, uint32_t* pop, uint32_t* bad,
                       hipStream_t s);
hipError_t launch_unpack(const ga_config* c, const uint32_t* pop, int8_t* q, hipStream_t s);

// ---- lanes per child (the children kernel's tile shape) -------------------
// 2, 4 or 8 for orders up to 32 (one word per column); 4 or 8 up to 64 (two
// words); 8 or 16 above (four words).
inline bool lanes_allowed(uint32_t m, uint32_t lanes) {
  if (m <= 32) return lanes == 2 || lanes == 4 || lanes == 8;
  if (m <= 64) return lanes == 4 || lanes == 8;
  return lanes == 8 || lanes == 16;
}
// The tuning table's choice for a launch of `children` children of order m.
uint32_t tuned_lanes(uint32_t m, uint64_t children);
// Forced lanes of a config (0 if the table decides).
inline uint32_t forced_lanes(const ga_config* c) {
  return (c->flags & GA_LANES_MASK) >> GA_LANES_SHIFT;
}
inline uint32_t children_per_block(uint32_t lanes) { return 64 / lanes; }

// ---- helpers (ga_api.hip) -----------------------------------------------
void set_error(const char* fmt, ...);
ga_status hip_status(hipError_t e, const char* what);
ga_status validate(const ga_config* c);
uint32_t words_per_col(uint32_t m);
PopDesc make_desc(const ga_config* c, uint32_t* pa, uint32_t* pb, uint32_t* ka,
                  uint32_t* kb, RunState* st, uint32_t max_gen,
                  uint32_t stop_on_found);
// Copies the best individual of a finished run into out (synchronous).
ga_status read_result(const ga_config* c, const RunState& hs,
                      const uint32_t* pop_a, const uint32_t* pop_b,
                      ga_result* out);

// ---- several independent runs advanced together (ga_multi.hip) ----------
// Device memory of one run: two populations, two key arrays.
struct RunBuffers {
  uint32_t* pop_a = nullptr;
  uint32_t* pop_b = nullptr;
  uint32_t* keys_a = nullptr;
  uint32_t* keys_b = nullptr;
  SelWork* sel = nullptr;  // runs with elitism or paper mode
  uint32_t* slots = nullptr;  // paper-mode runs: a chunk's slot table
  PaperWork* pw = nullptr;    // paper-mode runs up to kPaperTileMaxN with a table:
  uint32_t* psel = nullptr;   // the tile selection and its list (then slots holds pi)
  EliteWork* ew = nullptr;    // elitist runs: elites from candidate lists, as in
  uint32_t* earea = nullptr;  // ga_run (elite_area_words(n) words)
  void* base = nullptr;   // single allocation holding all of them
};
size_t run_bytes(const ga_config* c);
ga_status alloc_run(const ga_config* c, RunBuffers* b);
void free_run(RunBuffers* b);
// The launch descriptor of a batched or served run (with its selection
// workspace, if it selects).
PopDesc run_desc(const ga_config* c, const RunBuffers& b, RunState* st);

// Starts runs in place: state reset, initial population and its fitness.
ga_status start_runs(const ga_config* cfgs, const RunBuffers* bufs,
                     RunState* states, uint32_t count, hipStream_t s);

// Launch tables of a set of runs: one descriptor per run, and the map from
// a block of the children launch to its run, per group (one group per
// order).
class MultiLaunch {
 public:
  ~MultiLaunch();
  // descs: one per run (state pointers set); rebuilds and uploads the tables
  ga_status set(const PopDesc* descs, uint32_t count, hipStream_t s);
  // launch `node` of a chunk: one generation of every run still going
  // a chunk of `gens` launches and the gen_base advance, as one graph
  // launch on s (captured on first use after set(); s must not be the null
  // stream)
  ga_status launch_chunk(uint32_t gens, hipStream_t s);
  // the reported generation and best (key, slot) of every run
  ga_status finish(hipStream_t s);

 private:
  struct Group {
    uint32_t m = 0;                  // order
    uint32_t lanes = 0;              // lanes per child of the group's launch
    PopDesc* desc = nullptr;         // device tables read by the launches
    uint32_t* map = nullptr;
    PopDesc* hdesc = nullptr;        // pinned staging copies of the tables
    uint32_t* hmap = nullptr;
    size_t cap_desc = 0, cap_map = 0;
    uint32_t ndesc = 0, nblocks = 0;
    uint32_t npaper = 0;             // tile-selection blocks: map[nblocks ..], each
                                     // (run << 4 | tile)
    uint32_t nelite = 0;             // candidate-list elitist runs: map[nblocks +
                                     // npaper ..], each a run
  };
  // launch `node` for one group: its runs' selections (paper mode reading
  // row `node` of the slot tables when `tables`), then its children
  ga_status enqueue_group(const Group& g, uint32_t node, bool tables, hipStream_t s);
  Group groups_[kOrders];            // one per order 4, 8, .., 128
  hipGraphExec_t graph_ = nullptr;
  uint32_t graph_gens_ = 0;
  hipStream_t capture_ = nullptr;
  hipStream_t branch_[kOrders] = {};  // capture branches, one per group
  hipEvent_t fork_[kOrders + 1] = {};  // join events per group, fork event
};

}  // namespace ga
