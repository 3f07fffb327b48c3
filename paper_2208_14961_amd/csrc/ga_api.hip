// ga_api.hip -- the C ABI of libga (see include/ga.h): argument checks,
// per-stream device workspaces, and the orchestration of the kernels for
// single steps, whole runs and batches of runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "ga_internal.h"

namespace ga {

static thread_local std::string g_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
}

ga_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return GA_OK;
  set_error("%s: %s", what, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? GA_ENOMEM : GA_EDEVICE;
}

#define GA_TRY(expr, what)                          \
  do {                                              \
    ga_status _s = hip_status((expr), (what));      \
    if (_s != GA_OK) return _s;                     \
  } while (0)

uint32_t words_per_col(uint32_t m) { return col_words(m); }



ga_status validate(const ga_config* c) {
  if (!c) {
    set_error("config is NULL");
    return GA_EINVAL;
  }
  if (c->m < 4 || c->m > GA_MAX_M || c->m % 4) {
    set_error("m=%u: need m %% 4 == 0 and 4 <= m <= %u", c->m, (uint32_t)GA_MAX_M);
    return GA_EINVAL;
  }
  if (c->n < 2 || c->n > kMaxN) {
    set_error("n=%u: need 2 <= n <= %u", c->n, kMaxN);
    return GA_EINVAL;
  }
  if (c->max_generations > kMaxGenerations) {
    set_error("max_generations=%u: need at most %u", c->max_generations, kMaxGenerations);
    return GA_EINVAL;
  }
  if (c->fitness > GA_FIT_F2 || c->selection > GA_SEL_PAPER) {
    set_error("unknown fitness (%u) or selection (%u)", c->fitness,
              c->selection);
    return GA_EINVAL;
  }
  if (c->xo_threshold > (1ull << 32) || c->mut_threshold > (1ull << 32)) {
    set_error("coin thresholds must be <= 2^32");
    return GA_EINVAL;
  }
  if (c->nc > 64 || c->nr > 64 ||
      (c->mut_threshold > 0 && (c->nc == 0 || c->nr == 0))) {
    set_error("nc=%u nr=%u: need 1..64 when mutation is on", c->nc, c->nr);
    return GA_EINVAL;
  }
  if (c->flags & ~(uint32_t)(GA_STOP_ON_FOUND | GA_MUT_SHARED | GA_LANES_MASK | GA_GRAM_MASK)) {
    set_error("unknown flags 0x%x", c->flags);
    return GA_EINVAL;
  }
  const uint32_t gram = c->flags & GA_GRAM_MASK;
  if (gram == GA_GRAM_MASK || (gram == GA_GRAM_MFMA && c->m < kMfmaMinOrder)) {
    set_error("gram flags 0x%x: GA_GRAM_PACKED, or GA_GRAM_MFMA from order %u", gram,
              kMfmaMinOrder);
    return GA_EINVAL;
  }
  const uint32_t lanes = (c->flags & GA_LANES_MASK) >> GA_LANES_SHIFT;
  if (lanes != 0 && !lanes_allowed(c->m, lanes)) {
    set_error("lanes=%u: need 2, 4 or 8 for m <= 32, 4 or 8 for m <= 64, 8 or 16 above",
              lanes);
    return GA_EINVAL;
  }
  if (c->selection == GA_SEL_TOURNAMENT) {
    if (c->tournament_k < 1 || c->tournament_k > 64) {
      set_error("tournament_k=%u: need 1..64", c->tournament_k);
      return GA_EINVAL;
    }
    if (c->elite >= c->n || c->elite > kMaxElite) {
      set_error("elite=%u: need elite < n and elite <= %u", c->elite,
                kMaxElite);
      return GA_EINVAL;
    }
  } else if (c->n % 4 || c->elite) {
    set_error("paper mode: need n %% 4 == 0 and elite == 0");
    return GA_EINVAL;
  }
  const bool ranks = c->selection == GA_SEL_PAPER || c->elite > 0;
  if (ranks && max_key(c->m, c->fitness) >= (1ull << kKeyBits)) {
    set_error("m=%u: keys of fitness kind %u reach 2^%u, beyond what elitism and paper "
              "selection rank; use another kind or tournaments without elites",
              c->m, c->fitness, kKeyBits);
    return GA_EINVAL;
  }
  return GA_OK;
}

// Device workspace per (device, stream): the run state and the selection
// scratch.  Work enqueued on one stream is ordered, so it never races with
// itself; different streams get different workspaces.
struct Workspace {
  RunState* state = nullptr;
  SelWork* sel = nullptr;
  uint32_t* counter = nullptr;
  RunState* host_state = nullptr;  // pinned mirrors for polling (two slots)
  hipStream_t capture = nullptr;   // stream the generation graphs run on
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_t[2] = {nullptr, nullptr};  // timing of tuning chunks
  std::vector<hipEvent_t> ev_probe;  // around each timed children launch of the lanes measurement
  uint32_t* perm = nullptr;        // paper mode: a chunk's slot table
  uint64_t perm_cap = 0;           // its entries
  PaperWork* pw = nullptr;         // paper mode up to kPaperTileMaxN: the tile selection
  uint32_t* psel = nullptr;        // and its list of selected indices (psel_cap entries)
  uint64_t psel_cap = 0;
  // elitism: the next elites' sources, the candidate lists and the
  // selection's scratch, for populations up to elite_cap
  EliteWork* ew = nullptr;
  uint32_t* earea = nullptr;       // candidate lists and scratch (elite_area_words)
  uint64_t elite_cap = 0;
  // graphs of one chunk of generations, each valid for its key (the launch
  // descriptor, config and table); the last used last.  `graph` is the one
  // the last capture() chose.
  struct CachedGraph {
    std::vector<char> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<CachedGraph> graphs;
  hipGraphExec_t graph = nullptr;
};

// Graphs kept per workspace: the lanes-per-child candidates of one run shape.
constexpr size_t kGraphCache = 4;
// Runs of at least this many chunks measure the lanes-per-child candidates
// on their first kLanesRounds * candidates generations.
constexpr uint32_t kExploreMinChunks = 4;
constexpr uint32_t kLanesRounds = 8;
constexpr float kLanesMargin = 0.03f;

static hipError_t drop_graphs(Workspace* w) {
  hipError_t e = hipSuccess;
  for (auto& c : w->graphs)
    if (c.exec) {
      const hipError_t x = hipGraphExecDestroy(c.exec);
      if (e == hipSuccess) e = x;
    }
  w->graphs.clear();
  w->graph = nullptr;
  return e;
}

static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

static ga_status workspace(hipStream_t s, Workspace** out) {
  int dev = 0;
  GA_TRY(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto key = std::make_pair(dev, s);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) {
    *out = it->second;
    return GA_OK;
  }
  Workspace* w = new Workspace();
  GA_TRY(hipMalloc(&w->state, sizeof(RunState)), "hipMalloc(state)");
  GA_TRY(hipMalloc(&w->sel, sizeof(SelWork)), "hipMalloc(selection)");
  GA_TRY(hipMalloc(&w->counter, sizeof(uint32_t)), "hipMalloc(counter)");
  GA_TRY(hipHostMalloc(&w->host_state, 2 * sizeof(RunState),
                       hipHostMallocDefault),
         "hipHostMalloc(state)");
  GA_TRY(hipStreamCreateWithFlags(&w->capture, hipStreamNonBlocking),
         "hipStreamCreate");
  for (auto& e : w->ev)
    GA_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming),
           "hipEventCreate");
  for (auto& e : w->ev_t) GA_TRY(hipEventCreate(&e), "hipEventCreate");
  // the histograms start at zero (the kernels restore zeros); the memset
  // runs on the null stream, which later work on non-blocking streams does
  // not wait for, so wait for it here
  GA_TRY(hipMemset(w->sel, 0, sizeof(SelWork)), "hipMemset(selection)");
  GA_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  g_ws[key] = w;
  *out = w;
  return GA_OK;
}

PopDesc make_desc(const ga_config* c, uint32_t* pa, uint32_t* pb,
                         uint32_t* ka, uint32_t* kb, RunState* st,
                         uint32_t max_gen, uint32_t stop_on_found) {
  PopDesc d;
  memset(&d, 0, sizeof d);
  d.pop_a = pa;
  d.pop_b = pb;
  d.keys_a = ka;
  d.keys_b = kb;
  d.state = st;
  d.seed = c->seed;
  d.xo_thr = c->xo_threshold;
  d.mut_thr = c->mut_threshold;
  d.m = c->m;
  d.n = c->n;
  d.t = c->tournament_k;
  d.nc = c->nc;
  d.nr = c->nr;
  d.kind = c->fitness;
  d.paper = c->selection == GA_SEL_PAPER;
  if (d.paper) {
    d.elite = c->n / 2;   // offspring occupy slots 2N .. 4N-1
    d.nchild = c->n / 2;
  } else {
    d.elite = c->elite;
    d.nchild = c->n - c->elite;
  }
  d.max_gen = max_gen;
  d.stop_on_found = stop_on_found;
  d.block_begin = 0;
  d.lanes_forced = forced_lanes(c) ? 1u : 0u;
  d.mut_shared = (c->flags & GA_MUT_SHARED) ? 1u : 0u;
  d.lanes = forced_lanes(c) ? forced_lanes(c) : tuned_lanes(c->m, d.nchild);
  const uint32_t per_block = children_per_block(d.lanes);
  d.nblocks = (d.nchild + per_block - 1) / per_block;
  return d;
}

// Optional timing of ga_run's generation loop (ga_timing_*): HIP events on
// the loop's stream around the chunk launches; the mean is per generation.
struct Timing {
  bool on = false;
  hipEvent_t start = nullptr, stop = nullptr;
  double total_ms = 0;
  uint64_t gens = 0;
};
static Timing g_timing;

// Lanes per child measured by earlier runs, per launch shape.
struct TuneKey {
  uint32_t m, n, elite, kind, selection, t, nc, nr;
  bool operator<(const TuneKey& o) const {
    return std::tie(m, n, elite, kind, selection, t, nc, nr) <
           std::tie(o.m, o.n, o.elite, o.kind, o.selection, o.t, o.nc, o.nr);
  }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, uint32_t> g_tuned;

static TuneKey tune_key(const ga_config* c, const PopDesc&) {
  return TuneKey{c->m, c->n, c->elite, c->fitness, c->selection, c->tournament_k, c->nc, c->nr};
}
static bool tuned_lookup(const TuneKey& k, uint32_t* lanes) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(k);
  if (it == g_tuned.end()) return false;
  *lanes = it->second;
  return true;
}
static void tuned_store(const TuneKey& k, uint32_t lanes) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[k] = lanes;
}
static std::vector<uint32_t> lanes_candidates(uint32_t m) {
  if (m <= 32) return {2, 4, 8};
  if (m <= 64) return {4, 8};
  return {8, 16};
}
static void set_lanes(PopDesc* d, uint32_t lanes) {
  d->lanes = lanes;
  const uint32_t per = children_per_block(lanes);
  d->nblocks = (d->nchild + per - 1) / per;
}

static uint32_t select_count(const ga_config* c) {
  if (c->selection == GA_SEL_PAPER) return c->n / 2;
  return c->elite;
}

// Enqueues launch `node` of a chunk for a single population: the
// selection kernels if the mode needs them, then the children kernel.
// slots: paper mode's slot table row for this launch, or null.  With the
// elitism of ga_run (d.ew set) the children launch copies the elites chosen
// before it and one launch after it chooses the next generation's.
static ga_status enqueue_generation(const ga_config* c, const PopDesc& d,
                                    Workspace* w, uint32_t node,
                                    const uint32_t* slots, hipStream_t s) {
  if (d.ew) {
    GA_TRY(launch_children_one(d, node, s), "children kernel");
    GA_TRY(launch_elite_select(d, node + 1, s), "elite selection kernel");
    return GA_OK;
  }
  if (d.psel) {
    GA_TRY(launch_paper_select(d, node, d.psel, s), "selection kernels");
    GA_TRY(launch_children_one(d, node, s), "children kernel");
    return GA_OK;
  }
  const uint32_t cnt = select_count(c);
  if (cnt > 0)
    GA_TRY(launch_select(d, cnt, w->sel, node, slots, s), "selection kernels");
  GA_TRY(launch_children_one(d, node, s), "children kernel");
  return GA_OK;
}

static void unpack_matrix(uint32_t m, const uint32_t* words, int8_t* out) {
  const uint32_t W = words_per_col(m);
  memset(out, 0, (size_t)GA_MAX_M * GA_MAX_M);
  for (uint32_t r = 0; r < m; ++r)
    for (uint32_t j = 0; j < m; ++j) {
      const uint32_t bit = (words[j * W + r / 32] >> (r % 32)) & 1u;
      out[r * m + j] = bit ? -1 : 1;
    }
}

// Fills `out` from a finished run's state and its final buffers.
ga_status read_result(const ga_config* c, const RunState& hs,
                             const uint32_t* pop_a, const uint32_t* pop_b,
                             ga_result* out) {
  const uint32_t g = hs.final_gen;
  const unsigned long long b = hs.best;
  out->generation = g;
  out->best_key = (uint32_t)(b >> 32);
  out->index = (uint32_t)(b & 0xffffffffu);
  out->found = out->best_key == 0;
  const uint32_t mw = c->m * words_per_col(c->m);
  std::vector<uint32_t> words(mw);
  const uint32_t* src = ((g & 1u) ? pop_b : pop_a) + (size_t)out->index * mw;
  GA_TRY(hipMemcpy(words.data(), src, mw * sizeof(uint32_t),
                   hipMemcpyDeviceToHost),
         "hipMemcpy(best matrix)");
  unpack_matrix(c->m, words.data(), out->matrix);
  return GA_OK;
}

}  // namespace ga

using namespace ga;

extern "C" {

const char* ga_last_error(void) { return g_error.c_str(); }

ga_status ga_validate(const ga_config* cfg) { return validate(cfg); }

size_t ga_population_words(const ga_config* cfg) {
  if (validate(cfg) != GA_OK) return 0;
  return (size_t)cfg->n * cfg->m * words_per_col(cfg->m);
}

ga_status ga_init_population(const ga_config* cfg, uint32_t* pop,
                             void* stream) {
  ga_status st = validate(cfg);
  if (st != GA_OK) return st;
  if (!pop) {
    set_error("pop is NULL");
    return GA_EINVAL;
  }
  GA_TRY(launch_init(cfg, pop, (hipStream_t)stream), "init kernel");
  return GA_OK;
}

ga_status ga_fitness(const ga_config* cfg, const uint32_t* pop,
                     uint32_t* keys, uint32_t* comps, void* stream) {
  ga_status st = validate(cfg);
  if (st != GA_OK) return st;
  if (!pop || !keys) {
    set_error("pop or keys is NULL");
    return GA_EINVAL;
  }
  GA_TRY(launch_fitness(cfg, pop, keys, comps, nullptr, (hipStream_t)stream),
         "fitness kernel");
  return GA_OK;
}

uint32_t ga_tuned_lanes(const ga_config* cfg) {
  if (validate(cfg) != GA_OK) return 0;
  if (forced_lanes(cfg)) return forced_lanes(cfg);
  PopDesc d = make_desc(cfg, nullptr, nullptr, nullptr, nullptr, nullptr,
                        cfg->max_generations, 0);
  uint32_t known = 0;
  return tuned_lookup(tune_key(cfg, d), &known) ? known : d.lanes;
}

ga_status ga_fitness_repeat(const ga_config* cfg, const uint32_t* pop,
                            uint32_t* keys, uint32_t reps, void* stream) {
  ga_status st = validate(cfg);
  if (st != GA_OK) return st;
  if (!pop || !keys) {
    set_error("pop or keys is NULL");
    return GA_EINVAL;
  }
  if (reps == 0 || (uint64_t)cfg->n * reps >= (1ull << 40)) {
    set_error("reps=%u: need 1 <= reps and n * reps < 2^40", reps);
    return GA_EINVAL;
  }
  int dev = 0, cus = 0;
  GA_TRY(hipGetDevice(&dev), "hipGetDevice");
  GA_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
         "hipDeviceGetAttribute");
  GA_TRY(launch_fitness_repeat(cfg, pop, keys, reps, (uint32_t)cus,
                               (hipStream_t)stream),
         "fitness kernel");
  return GA_OK;
}

ga_status ga_step(const ga_config* cfg, const uint32_t* pop_in,
                  const uint32_t* keys_in, uint32_t* pop_out,
                  uint32_t* keys_out, uint32_t gen_in, void* stream) {
  ga_status st = validate(cfg);
  if (st != GA_OK) return st;
  if (!pop_in || !keys_in || !pop_out || !keys_out || pop_in == pop_out ||
      keys_in == keys_out) {
    set_error("ga_step needs four distinct non-NULL buffers");
    return GA_EINVAL;
  }
  if (gen_in == 0xffffffffu) {
    set_error("gen_in too large");
    return GA_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  Workspace* w;
  st = workspace(s, &w);
  if (st != GA_OK) return st;
  // generation g lives in the "a" buffers iff g is even
  uint32_t* pi = const_cast<uint32_t*>(pop_in);
  uint32_t* ki = const_cast<uint32_t*>(keys_in);
  const bool odd = gen_in & 1u;
  PopDesc d = make_desc(cfg, odd ? pop_out : pi, odd ? pi : pop_out,
                        odd ? keys_out : ki, odd ? ki : keys_out, w->state,
                        0xffffffffu, 0);
  GA_TRY(launch_set_state(w->state, gen_in, s), "state kernel");
  return enqueue_generation(cfg, d, w, 0, nullptr, s);
}

ga_status ga_paper_select(const ga_config* cfg, const uint32_t* keys, uint32_t* threshold,
                          uint32_t* sel, void* stream) {
  ga_status st = validate(cfg);
  if (st != GA_OK) return st;
  if (cfg->selection != GA_SEL_PAPER || cfg->n > kPaperTileMaxN) {
    set_error("ga_paper_select: need paper mode and n <= %u", kPaperTileMaxN);
    return GA_EINVAL;
  }
  if (!keys || !threshold || !sel) {
    set_error("ga_paper_select needs non-NULL buffers");
    return GA_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  Workspace* w;
  st = workspace(s, &w);
  if (st != GA_OK) return st;
  if (!w->pw) {
    GA_TRY(hipMalloc(&w->pw, sizeof(PaperWork)), "hipMalloc(selection)");
    GA_TRY(hipMemset(w->pw, 0, sizeof(PaperWork)), "hipMemset(selection)");
  }
  uint32_t* k = const_cast<uint32_t*>(keys);
  // the selection of generation 1's parents: the keys are generation 0's
  PopDesc d = make_desc(cfg, nullptr, nullptr, k, k, w->state, 1, 0);
  d.pw = w->pw;
  GA_TRY(launch_set_state(w->state, 0, s), "state kernel");
  // generation 1's selection reads T[0] and writes T[1]
  GA_TRY(hipMemcpyAsync(&w->pw->T[0], threshold, sizeof(uint32_t), hipMemcpyDeviceToDevice, s),
         "hipMemcpyAsync(threshold)");
  GA_TRY(launch_paper_select(d, 0, sel, s), "selection kernels");
  GA_TRY(hipMemcpyAsync(threshold, &w->pw->T[1], sizeof(uint32_t), hipMemcpyDeviceToDevice, s),
         "hipMemcpyAsync(threshold)");
  return GA_OK;
}

ga_status ga_run(const ga_config* cfg, uint32_t* pop_a, uint32_t* pop_b,
                 uint32_t* keys_a, uint32_t* keys_b, ga_result* out,
                 void* stream) {
  ga_status st = validate(cfg);
  if (st != GA_OK) return st;
  if (!pop_a || !pop_b || !keys_a || !keys_b || !out || pop_a == pop_b ||
      keys_a == keys_b) {
    set_error("ga_run needs distinct non-NULL buffers and a result");
    return GA_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  Workspace* w;
  st = workspace(s, &w);
  if (st != GA_OK) return st;
  const uint32_t stop_on_found = (cfg->flags & GA_STOP_ON_FOUND) ? 1u : 0u;
  PopDesc d = make_desc(cfg, pop_a, pop_b, keys_a, keys_b, w->state,
                        cfg->max_generations, stop_on_found);
  GA_TRY(launch_reset_state(w->state, s), "state kernel");
  GA_TRY(launch_init(cfg, pop_a, s), "init kernel");
  GA_TRY(launch_fitness(cfg, pop_a, keys_a, nullptr, w->state, s),
         "fitness kernel");
  // Generations run in chunks: one captured graph of `chunk` launches and
  // the gen_base advance, replayed.  The host reads the state of chunk k
  // while chunk k+1 runs; launches past the end of the run return at once.
  const uint32_t chunk = std::min<uint32_t>(64, std::max<uint32_t>(1, cfg->max_generations));
  const uint32_t nchunks = (uint32_t)(((uint64_t)cfg->max_generations + chunk - 1) / chunk);
  // Paper mode: the chunk's slot permutations are computed by one launch at
  // its start (when the table stays small), not inside each scatter.
  const uint32_t D = cfg->selection == GA_SEL_PAPER ? cfg->n / 2 : 0;
  const bool table = D > 0 && nchunks > 0 && (uint64_t)D * chunk <= kMaxPermTable;
  if (table && w->perm_cap < (uint64_t)D * chunk) {
    // a cached graph may still run with the old table
    GA_TRY(hipStreamSynchronize(w->capture), "hipStreamSynchronize");
    GA_TRY(drop_graphs(w), "hipGraphExecDestroy");
    if (w->perm) GA_TRY(hipFree(w->perm), "hipFree(slot table)");
    w->perm = nullptr;
    w->perm_cap = 0;
    GA_TRY(hipMalloc(&w->perm, (size_t)D * chunk * sizeof(uint32_t)), "hipMalloc(slot table)");
    w->perm_cap = (uint64_t)D * chunk;
  }
  // Elitism: the elites come from a short candidate list each generation
  // (EliteWork), on buffers sized for the population.
  const bool elites = cfg->selection == GA_SEL_TOURNAMENT && cfg->elite > 0 && nchunks > 0;
  if (elites && w->elite_cap < cfg->n) {
    GA_TRY(hipStreamSynchronize(w->capture), "hipStreamSynchronize");
    GA_TRY(drop_graphs(w), "hipGraphExecDestroy");
    if (w->earea) GA_TRY(hipFree(w->earea), "hipFree(candidate lists)");
    w->earea = nullptr;
    w->elite_cap = 0;
    if (!w->ew) GA_TRY(hipMalloc(&w->ew, sizeof(EliteWork)), "hipMalloc(elites)");
    GA_TRY(hipMalloc(&w->earea, elite_area_words(cfg->n) * sizeof(uint32_t)),
           "hipMalloc(candidate lists)");
    w->elite_cap = cfg->n;
  }
  if (elites) {
    d.ew = w->ew;
    set_elite_area(&d, w->earea);
  }
  // Paper mode up to kPaperOneBlockMaxN: one block selects (indices and
  // keys into psel) and the children launch gathers the parents through the
  // chunk's forward slot table.
  const bool tiles = table && cfg->n <= kPaperTileMaxN;
  if (tiles && !w->pw) {
    GA_TRY(hipMalloc(&w->pw, sizeof(PaperWork)), "hipMalloc(selection)");
    GA_TRY(hipMemset(w->pw, 0, sizeof(PaperWork)), "hipMemset(selection)");
  }
  if (tiles && w->psel_cap < D) {
    GA_TRY(hipStreamSynchronize(w->capture), "hipStreamSynchronize");
    GA_TRY(drop_graphs(w), "hipGraphExecDestroy");
    if (w->psel) GA_TRY(hipFree(w->psel), "hipFree(selected list)");
    w->psel = nullptr;
    w->psel_cap = 0;
    GA_TRY(hipMalloc(&w->psel, (size_t)D * sizeof(uint32_t)), "hipMalloc(selected list)");
    w->psel_cap = D;
  }
  if (tiles) {  // the chunk's table holds pi (forward) for the children launches
    d.pw = w->pw;
    d.psel = w->psel;
    d.pfwd = w->perm;
  }
  auto capture = [&](const PopDesc& dd) -> ga_status {
    std::vector<char> key(sizeof(PopDesc) + sizeof(ga_config) + sizeof(uint32_t*));
    uint32_t* tab = table ? w->perm : nullptr;
    memcpy(key.data(), &dd, sizeof(PopDesc));
    memcpy(key.data() + sizeof(PopDesc), cfg, sizeof(ga_config));
    memcpy(key.data() + sizeof(PopDesc) + sizeof(ga_config), &tab, sizeof tab);
    for (size_t i = 0; i < w->graphs.size(); ++i)
      if (w->graphs[i].key == key) {  // most recently used last
        Workspace::CachedGraph c = std::move(w->graphs[i]);
        w->graphs.erase(w->graphs.begin() + i);
        w->graphs.push_back(std::move(c));
        w->graph = w->graphs.back().exec;
        return GA_OK;
      }
    if (w->graphs.size() >= kGraphCache) {
      GA_TRY(hipGraphExecDestroy(w->graphs.front().exec), "hipGraphExecDestroy");
      w->graphs.erase(w->graphs.begin());
    }
    w->graph = nullptr;
    hipGraph_t g;
    GA_TRY(hipStreamBeginCapture(w->capture, hipStreamCaptureModeThreadLocal),
           "hipStreamBeginCapture");
    ga_status cs = GA_OK;
    if (tab)
      cs = hip_status(launch_perm_table(dd, D, chunk, tab, w->capture, dd.psel != nullptr),
                      "slot table kernel");
    for (uint32_t i = 0; i < chunk && cs == GA_OK; ++i)
      cs = enqueue_generation(cfg, dd, w, i, tab ? tab + (size_t)i * D : nullptr, w->capture);
    if (cs == GA_OK)
      cs = hip_status(launch_advance_one(w->state, chunk, w->capture), "advance kernel");
    hipError_t ce = hipStreamEndCapture(w->capture, &g);
    if (cs != GA_OK) return cs;
    GA_TRY(ce, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    GA_TRY(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    GA_TRY(hipGraphDestroy(g), "hipGraphDestroy");
    w->graphs.push_back(Workspace::CachedGraph{key, exec});
    w->graph = exec;
    return GA_OK;
  };
  // Lanes per child: forced by the config, or measured at the start of the
  // run and remembered for later runs of the same shape, or, for runs too
  // short for the measurement to pay, the tuning table's.
  const TuneKey tkey = tune_key(cfg, d);
  const std::vector<uint32_t> cands = lanes_candidates(cfg->m);
  bool explore = false;
  const uint32_t table_lanes = d.lanes;  // the tuning table's choice
  if (!forced_lanes(cfg)) {
    uint32_t known = 0;
    if (tuned_lookup(tkey, &known)) set_lanes(&d, known);
    else explore = nchunks >= kExploreMinChunks;
  }
  if (nchunks > 0) {
    // the capture stream starts after the work already enqueued on s
    GA_TRY(hipEventRecord(w->ev[2], s), "hipEventRecord");
    GA_TRY(hipStreamWaitEvent(w->capture, w->ev[2], 0), "hipStreamWaitEvent");
    // the first generation's elites, from the whole initial population, and
    // empty candidate lists
    if (elites) {
      GA_TRY(hipMemsetAsync(d.ecount, 0, kEliteLists * sizeof(uint32_t), w->capture),
             "hipMemsetAsync(candidate lists)");
      GA_TRY(launch_select(d, cfg->elite, w->sel, 0, nullptr, w->capture, w->ew->src,
                           &w->ew->kstar),
             "selection kernels");
    }
    // no earlier threshold: the first selection searches every key
    if (tiles) {
      GA_TRY(hipMemsetAsync(w->pw->T, 0xff, sizeof(w->pw->T), w->capture),
             "hipMemsetAsync(selection)");
    }
  }
  uint32_t probed = 0;      // generations made by the lanes measurement
  bool ended = false;       // the run ended inside them
  if (explore) {
    // The run's first generations, launched one by one from the stream,
    // each with the next candidate (rounds in the order c1 .. ck, ck .. c1,
    // c1 .. ck, ...), every children launch between two events.  Every
    // variant makes the same generations, so the run's results do not depend
    // on the measurement; each candidate is timed on fresh generations (their
    // inputs written by the launch before, as in the chunks) next to the
    // others, so the cost's drift over the run (the selection's changes as
    // the population converges) weighs on all alike.  Each candidate counts
    // the median of its launches after the first round; the tuning table's
    // choice (timed on whole runs of the same order and size) stays unless
    // another candidate is faster by more than kLanesMargin.
    const uint32_t nc = (uint32_t)cands.size();
    const uint32_t K = kLanesRounds * nc;
    while (w->ev_probe.size() < 2 * (size_t)K) {
      hipEvent_t e;
      GA_TRY(hipEventCreate(&e), "hipEventCreate");
      w->ev_probe.push_back(e);
    }
    const uint32_t cnt = select_count(cfg);
    if (table)
      GA_TRY(launch_perm_table(d, D, K, w->perm, w->capture, d.psel != nullptr),
             "slot table kernel");
    std::vector<uint32_t> who(K);
    for (uint32_t node = 0; node < K; ++node) {
      const uint32_t round = node / nc, pos = node % nc;
      const uint32_t ci = (round & 1u) ? nc - 1 - pos : pos;
      who[node] = ci;
      PopDesc dc = d;
      set_lanes(&dc, cands[ci]);
      if (dc.psel) {
        GA_TRY(launch_paper_select(dc, node, dc.psel, w->capture), "selection kernels");
      } else if (!dc.ew && cnt > 0) {
        GA_TRY(launch_select(dc, cnt, w->sel, node, table ? w->perm + (size_t)node * D : nullptr,
                             w->capture),
               "selection kernels");
      }
      GA_TRY(hipEventRecord(w->ev_probe[2 * node], w->capture), "hipEventRecord");
      GA_TRY(launch_children_one(dc, node, w->capture), "children kernel");
      GA_TRY(hipEventRecord(w->ev_probe[2 * node + 1], w->capture), "hipEventRecord");
      if (dc.ew) GA_TRY(launch_elite_select(dc, node + 1, w->capture), "elite selection kernel");
    }
    GA_TRY(launch_advance_one(w->state, K, w->capture), "advance kernel");
    GA_TRY(hipMemcpyAsync(&w->host_state[0], w->state, sizeof(RunState), hipMemcpyDeviceToHost,
                          w->capture),
           "hipMemcpyAsync(state)");
    GA_TRY(hipStreamSynchronize(w->capture), "hipStreamSynchronize");
    std::vector<std::vector<float>> ms(nc);
    for (uint32_t node = nc; node < K; ++node) {
      float t = 0;
      GA_TRY(hipEventElapsedTime(&t, w->ev_probe[2 * node], w->ev_probe[2 * node + 1]),
             "hipEventElapsedTime");
      ms[who[node]].push_back(t);
    }
    uint32_t best = 0;
    float best_t = 0;
    std::vector<float> med(nc);
    for (uint32_t ci = 0; ci < nc; ++ci) {
      std::vector<float>& v = ms[ci];
      std::sort(v.begin(), v.end());
      med[ci] = v[v.size() / 2];
      if (ci == 0 || med[ci] < best_t) {
        best = ci;
        best_t = med[ci];
      }
    }
    for (uint32_t ci = 0; ci < nc; ++ci)
      if (cands[ci] == table_lanes && best_t > (1.f - kLanesMargin) * med[ci]) best = ci;
    probed = K;
    // a run that ended inside the measured generations (launches after its
    // end return at once) measured nothing
    ended = run_done(w->host_state[0], cfg->max_generations, stop_on_found);
    if (!ended) tuned_store(tkey, cands[best]);
    set_lanes(&d, cands[best]);
  }
  // chunks for the generations after the measured ones
  const uint32_t rest = ended || probed >= cfg->max_generations
                            ? 0u
                            : (uint32_t)(((uint64_t)cfg->max_generations - probed + chunk - 1) / chunk);
  if (rest > 0) {
    st = capture(d);
    if (st != GA_OK) return st;
    // the capture stream starts after the work already enqueued on s
    GA_TRY(hipEventRecord(w->ev[2], s), "hipEventRecord");
    GA_TRY(hipStreamWaitEvent(w->capture, w->ev[2], 0), "hipStreamWaitEvent");
    if (g_timing.on) GA_TRY(hipEventRecord(g_timing.start, w->capture), "hipEventRecord");
    auto launch_chunk = [&](uint32_t k) -> ga_status {
      GA_TRY(hipGraphLaunch(w->graph, w->capture), "hipGraphLaunch");
      GA_TRY(hipMemcpyAsync(&w->host_state[k & 1], w->state, sizeof(RunState),
                            hipMemcpyDeviceToHost, w->capture),
             "hipMemcpyAsync(state)");
      GA_TRY(hipEventRecord(w->ev[k & 1], w->capture), "hipEventRecord");
      return GA_OK;
    };
    st = launch_chunk(0);
    if (st != GA_OK) return st;
    for (uint32_t k = 0; k < rest; ++k) {
      if (k + 1 < rest) {
        st = launch_chunk(k + 1);
        if (st != GA_OK) return st;
      }
      GA_TRY(hipEventSynchronize(w->ev[k & 1]), "hipEventSynchronize");
      if (run_done(w->host_state[k & 1], cfg->max_generations, stop_on_found))
        break;
    }
    if (g_timing.on) {
      // the chunks launched after the stop condition return at once; the
      // mean is over the generations made inside the timed chunks
      GA_TRY(hipEventRecord(g_timing.stop, w->capture), "hipEventRecord");
      GA_TRY(hipEventSynchronize(g_timing.stop), "hipEventSynchronize");
      float ms = 0;
      GA_TRY(hipEventElapsedTime(&ms, g_timing.start, g_timing.stop),
             "hipEventElapsedTime");
      const RunState& hs = w->host_state[0].gen_base >= w->host_state[1].gen_base
                               ? w->host_state[0] : w->host_state[1];
      uint32_t made = std::min(cfg->max_generations, hs.gen_base);
      if (stop_on_found && hs.found_gen < made) made = hs.found_gen;
      g_timing.total_ms += ms;
      g_timing.gens += made > probed ? made - probed : 0;
    }
  }
  if (nchunks > 0) {
    // s continues after everything the capture stream did
    GA_TRY(hipEventRecord(w->ev[2], w->capture), "hipEventRecord");
    GA_TRY(hipStreamWaitEvent(s, w->ev[2], 0), "hipStreamWaitEvent");
  }
  GA_TRY(launch_finish_one(d, s), "finish kernel");
  GA_TRY(hipMemcpyAsync(w->host_state, w->state, sizeof(RunState),
                        hipMemcpyDeviceToHost, s),
         "hipMemcpyAsync(state)");
  GA_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  RunState hs = *w->host_state;
  return read_result(cfg, hs, pop_a, pop_b, out);
}

ga_status ga_timing_enable(int on) {
  if (on && !g_timing.start) {
    GA_TRY(hipEventCreate(&g_timing.start), "hipEventCreate");
    GA_TRY(hipEventCreate(&g_timing.stop), "hipEventCreate");
  }
  g_timing.on = on != 0;
  if (g_timing.on) {
    g_timing.total_ms = 0;
    g_timing.gens = 0;
  }
  return GA_OK;
}

ga_status ga_timing_read(double* mean_ms, uint64_t* launches) {
  if (!mean_ms || !launches) {
    set_error("ga_timing_read needs two outputs");
    return GA_EINVAL;
  }
  *launches = g_timing.gens;
  *mean_ms = g_timing.gens ? g_timing.total_ms / (double)g_timing.gens : 0.0;
  return GA_OK;
}

ga_status ga_pack(const ga_config* cfg, const int8_t* q, uint32_t* pop,
                  uint32_t* bad, void* stream) {
  ga_status st = validate(cfg);
  if (st != GA_OK) return st;
  if (!q || !pop) {
    set_error("q or pop is NULL");
    return GA_EINVAL;
  }
  GA_TRY(launch_pack(cfg, q, pop, bad, (hipStream_t)stream), "pack kernel");
  return GA_OK;
}

ga_status ga_unpack(const ga_config* cfg, const uint32_t* pop, int8_t* q,
                    void* stream) {
  ga_status st = validate(cfg);
  if (st != GA_OK) return st;
  if (!q || !pop) {
    set_error("q or pop is NULL");
    return GA_EINVAL;
  }
  GA_TRY(launch_unpack(cfg, pop, q, (hipStream_t)stream), "unpack kernel");
  return GA_OK;
}

ga_status ga_check_invariants(const ga_config* cfg, const uint32_t* pop,
                              uint32_t* bad_count, void* stream) {
  ga_status st = validate(cfg);
  if (st != GA_OK) return st;
  if (!pop || !bad_count) {
    set_error("pop or bad_count is NULL");
    return GA_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  Workspace* w;
  st = workspace(s, &w);
  if (st != GA_OK) return st;
  GA_TRY(hipMemsetAsync(w->counter, 0, sizeof(uint32_t), s), "hipMemsetAsync");
  GA_TRY(launch_check(cfg, pop, w->counter, s), "check kernel");
  GA_TRY(hipMemcpyAsync(bad_count, w->counter, sizeof(uint32_t),
                        hipMemcpyDeviceToHost, s),
         "hipMemcpyAsync");
  GA_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return GA_OK;
}

}  // extern "C"
