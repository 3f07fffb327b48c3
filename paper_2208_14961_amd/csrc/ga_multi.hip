// ga_multi.hip -- several independent runs advanced one generation per
// launch: the batched entry point ga_run_batch and the building blocks the
// search server shares with it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ga_common.h"

namespace ga {

#define GA_TRY(expr, what)                          \
  do {                                              \
    ga_status _s = hip_status((expr), (what));      \
    if (_s != GA_OK) return _s;                     \
  } while (0)

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Elitism and paper mode select every generation; such a run carries its
// own selection workspace.
static bool selects(const ga_config* c) {
  return c->selection == GA_SEL_PAPER || c->elite > 0;
}

// Paper-mode runs whose chunk table stays small get one (the batched graph
// computes a chunk's slot permutations in one launch, as ga_run does).
static size_t table_bytes(const ga_config* c) {
  if (c->selection != GA_SEL_PAPER) return 0;
  const uint64_t entries = (uint64_t)(c->n / 2) * kBatchTableRows;
  return entries <= kMaxPermTable ? align256(entries * sizeof(uint32_t)) : 0;
}

// Paper-mode runs with a table and at most kPaperTileMaxN individuals select
// as ga_run does (ga_paper.hip); their table then holds pi, not pi^-1.
static size_t tile_bytes(const ga_config* c) {
  if (!table_bytes(c) || c->n > kPaperTileMaxN) return 0;
  return align256(sizeof(PaperWork)) + align256((size_t)(c->n / 2) * sizeof(uint32_t));
}

// Elitist runs choose their elites as ga_run does: from the previous elites
// and the children listed below the largest elite key (ga_elite.hip).
static size_t elite_bytes(const ga_config* c) {
  if (c->selection != GA_SEL_TOURNAMENT || c->elite == 0) return 0;
  return align256(sizeof(EliteWork)) + align256(elite_area_words(c->n) * 4);
}

size_t run_bytes(const ga_config* c) {
  const size_t pop = (size_t)c->n * c->m * words_per_col(c->m) * 4;
  const size_t keys = (size_t)c->n * 4;
  return 2 * align256(pop) + 2 * align256(keys) + (selects(c) ? align256(sizeof(SelWork)) : 0) +
         table_bytes(c) + tile_bytes(c) + elite_bytes(c);
}

ga_status alloc_run(const ga_config* c, RunBuffers* b) {
  const size_t pop = align256((size_t)c->n * c->m * words_per_col(c->m) * 4);
  const size_t keys = align256((size_t)c->n * 4);
  char* base = nullptr;
  GA_TRY(hipMalloc(&base, run_bytes(c)), "hipMalloc(run)");
  b->base = base;
  b->pop_a = reinterpret_cast<uint32_t*>(base);
  b->pop_b = reinterpret_cast<uint32_t*>(base + pop);
  b->keys_a = reinterpret_cast<uint32_t*>(base + 2 * pop);
  b->keys_b = reinterpret_cast<uint32_t*>(base + 2 * pop + keys);
  const size_t sel = selects(c) ? align256(sizeof(SelWork)) : 0;
  b->sel = sel ? reinterpret_cast<SelWork*>(base + 2 * pop + 2 * keys) : nullptr;
  b->slots = table_bytes(c) ? reinterpret_cast<uint32_t*>(base + 2 * pop + 2 * keys + sel)
                            : nullptr;
  if (tile_bytes(c)) {
    char* t = base + 2 * pop + 2 * keys + sel + table_bytes(c);
    b->pw = reinterpret_cast<PaperWork*>(t);
    b->psel = reinterpret_cast<uint32_t*>(t + align256(sizeof(PaperWork)));
  }
  if (elite_bytes(c)) {
    char* t = base + 2 * pop + 2 * keys + sel + table_bytes(c) + tile_bytes(c);
    b->ew = reinterpret_cast<EliteWork*>(t);
    t += align256(sizeof(EliteWork));
    b->earea = reinterpret_cast<uint32_t*>(t);
  }
  return GA_OK;
}

PopDesc run_desc(const ga_config* c, const RunBuffers& b, RunState* st) {
  PopDesc d = make_desc(c, b.pop_a, b.pop_b, b.keys_a, b.keys_b, st, c->max_generations,
                        (c->flags & GA_STOP_ON_FOUND) ? 1u : 0u);
  d.sel = b.sel;
  d.slots = b.slots;
  if (b.pw) {
    d.pw = b.pw;
    d.psel = b.psel;
    d.pfwd = b.slots;
  }
  if (b.ew) {
    d.ew = b.ew;
    set_elite_area(&d, b.earea);
  }
  return d;
}

void free_run(RunBuffers* b) {
  if (b->base) (void)hipFree(b->base);
  *b = RunBuffers();
}

MultiLaunch::~MultiLaunch() {
  if (graph_) (void)hipGraphExecDestroy(graph_);
  if (capture_) {
    (void)hipStreamDestroy(capture_);
    for (auto b : branch_)
      if (b) (void)hipStreamDestroy(b);
    for (auto e : fork_) (void)hipEventDestroy(e);
  }
  for (Group& g : groups_) {
    if (g.desc) (void)hipFree(g.desc);
    if (g.map) (void)hipFree(g.map);
    if (g.hdesc) (void)hipHostFree(g.hdesc);
    if (g.hmap) (void)hipHostFree(g.hmap);
  }
}

static int group_of(uint32_t m) { return (int)(m / 4) - 1; }

ga_status MultiLaunch::set(const PopDesc* descs, uint32_t count,
                           hipStream_t s) {
  // s idle: no earlier copy still reads the staging buffers and no earlier
  // launch still reads the device tables
  GA_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (graph_) {
    GA_TRY(hipGraphExecDestroy(graph_), "hipGraphExecDestroy");
    graph_ = nullptr;
  }
  for (int gi = 0; gi < kOrders; ++gi) {
    Group& g = groups_[gi];
    g.m = 4u * (gi + 1);
    std::vector<PopDesc> ds;
    std::vector<uint32_t> map;
    // one lanes-per-child choice per group: forced by a run's config if any
    // run of the order forces it, else the tuning table's for the group's
    // total children (they share one launch)
    uint64_t children = 0;
    uint32_t forced = 0;
    for (uint32_t i = 0; i < count; ++i) {
      if (group_of(descs[i].m) != gi) continue;
      children += descs[i].nchild;
      if (!forced && descs[i].lanes_forced) forced = descs[i].lanes;
    }
    g.lanes = forced ? forced : (children ? tuned_lanes(g.m, children) : 0);
    for (uint32_t i = 0; i < count; ++i) {
      if (group_of(descs[i].m) != gi) continue;
      PopDesc d = descs[i];
      d.lanes = g.lanes;
      d.nblocks = (d.nchild + children_per_block(g.lanes) - 1) / children_per_block(g.lanes);
      d.block_begin = (uint32_t)map.size();
      for (uint32_t b = 0; b < d.nblocks; ++b)
        map.push_back((uint32_t)ds.size());
      ds.push_back(d);
    }
    g.nblocks = (uint32_t)map.size();
    g.ndesc = (uint32_t)ds.size();
    // the tile selection's blocks of the group's paper-mode runs follow
    for (uint32_t j = 0; j < ds.size(); ++j)
      if (ds[j].pw)
        for (uint32_t t = 0; t < (ds[j].n + kPaperTile - 1) / kPaperTile; ++t)
          map.push_back(j << 4 | t);
    g.npaper = (uint32_t)map.size() - g.nblocks;
    // then the group's candidate-list elitist runs
    for (uint32_t j = 0; j < ds.size(); ++j)
      if (ds[j].ew) map.push_back(j);
    g.nelite = (uint32_t)map.size() - g.nblocks - g.npaper;
    if (ds.empty()) continue;
    // The launches on s read these tables, so they are uploaded on s itself
    // (stream order puts the copy before the launches) from pinned staging
    // memory.
    if (ds.size() > g.cap_desc) {
      if (g.desc) GA_TRY(hipFree(g.desc), "hipFree");
      if (g.hdesc) GA_TRY(hipHostFree(g.hdesc), "hipHostFree");
      g.desc = nullptr;
      g.hdesc = nullptr;
      g.cap_desc = ds.size() * 2;
      GA_TRY(hipMalloc(&g.desc, g.cap_desc * sizeof(PopDesc)), "hipMalloc(descs)");
      GA_TRY(hipHostMalloc(&g.hdesc, g.cap_desc * sizeof(PopDesc), hipHostMallocDefault),
             "hipHostMalloc(descs)");
    }
    if (map.size() > g.cap_map) {
      if (g.map) GA_TRY(hipFree(g.map), "hipFree");
      if (g.hmap) GA_TRY(hipHostFree(g.hmap), "hipHostFree");
      g.map = nullptr;
      g.hmap = nullptr;
      g.cap_map = map.size() * 2;
      GA_TRY(hipMalloc(&g.map, g.cap_map * sizeof(uint32_t)), "hipMalloc(block map)");
      GA_TRY(hipHostMalloc(&g.hmap, g.cap_map * sizeof(uint32_t), hipHostMallocDefault),
             "hipHostMalloc(block map)");
    }
    memcpy(g.hdesc, ds.data(), ds.size() * sizeof(PopDesc));
    memcpy(g.hmap, map.data(), map.size() * sizeof(uint32_t));
    GA_TRY(hipMemcpyAsync(g.desc, g.hdesc, ds.size() * sizeof(PopDesc),
                          hipMemcpyHostToDevice, s),
           "hipMemcpyAsync(descs)");
    GA_TRY(hipMemcpyAsync(g.map, g.hmap, map.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice, s),
           "hipMemcpyAsync(block map)");
  }
  return GA_OK;
}

// Launch `node` of a chunk for one order group: the selections of its runs
// that select (elitism, paper mode; each on its own workspace), then the
// group's children launch.
ga_status MultiLaunch::enqueue_group(const Group& g, uint32_t node, bool tables,
                                     hipStream_t s) {
  if (g.npaper) {  // every tile-selecting run of the group in two launches
    if (!tables) {  // their children launch reads the chunk's table of pi
      set_error("internal: a tile-selecting run without its chunk table");
      return GA_EINVAL;
    }
    GA_TRY(launch_paper_select_multi(g.desc, g.map + g.nblocks, g.npaper, node, s),
           "selection kernels");
  }
  for (uint32_t i = 0; i < g.ndesc; ++i) {
    const PopDesc& d = g.hdesc[i];
    if (d.pw || d.ew || !d.sel) continue;
    const uint32_t* row =
        (tables && d.paper && d.slots) ? d.slots + (size_t)node * (d.n / 2) : nullptr;
    GA_TRY(launch_select(d, d.paper ? d.n / 2 : d.elite, d.sel, node, row, s),
           "selection kernels");
  }
  GA_TRY(launch_children(g.desc, g.map, g.nblocks, g.m, g.lanes, node, s),
         "children kernel");
  // the elites of the next generation, from the elites and the marked children
  if (g.nelite)
    GA_TRY(launch_elite_select_multi(g.desc, g.map + g.nblocks + g.npaper, g.nelite, node + 1, s),
           "elite selection kernel");
  return GA_OK;
}

ga_status MultiLaunch::finish(hipStream_t s) {
  for (Group& g : groups_)
    if (g.ndesc) GA_TRY(launch_finish(g.desc, g.ndesc, s), "finish kernel");
  return GA_OK;
}

// The chunk graph holds one independent chain per order group (a group's
// generation G depends only on its own generation G - 1): the capture forks
// one stream per group from the capture stream and joins them at the end,
// so the groups' launches may run side by side.
ga_status MultiLaunch::launch_chunk(uint32_t gens, hipStream_t s) {
  if (!graph_ || graph_gens_ != gens) {
    if (graph_) {
      GA_TRY(hipGraphExecDestroy(graph_), "hipGraphExecDestroy");
      graph_ = nullptr;
    }
    if (!capture_) {
      GA_TRY(hipStreamCreateWithFlags(&capture_, hipStreamNonBlocking),
             "hipStreamCreate");
      for (auto& e : fork_)
        GA_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming),
               "hipEventCreate");
    }
    // a capture branch only for the orders in use
    for (int gi = 0; gi < kOrders; ++gi)
      if (groups_[gi].ndesc && !branch_[gi])
        GA_TRY(hipStreamCreateWithFlags(&branch_[gi], hipStreamNonBlocking),
               "hipStreamCreate");
    hipGraph_t g;
    GA_TRY(hipStreamBeginCapture(capture_, hipStreamCaptureModeThreadLocal),
           "hipStreamBeginCapture");
    ga_status st = hip_status(hipEventRecord(fork_[kOrders], capture_), "hipEventRecord");
    for (int gi = 0; gi < kOrders && st == GA_OK; ++gi) {
      Group& gr = groups_[gi];
      if (!gr.ndesc) continue;
      hipStream_t b = branch_[gi];
      st = hip_status(hipStreamWaitEvent(b, fork_[kOrders], 0), "hipStreamWaitEvent");
      // paper-mode runs: the chunk's slot permutations first, in one launch each
      const bool tables = gens <= kBatchTableRows;
      for (uint32_t j = 0; j < gr.ndesc && st == GA_OK && tables; ++j) {
        const PopDesc& d = gr.hdesc[j];
        if (d.paper && d.slots)
          st = hip_status(launch_perm_table(d, d.n / 2, gens, d.slots, b, d.pw != nullptr),
                          "slot table kernel");
      }
      for (uint32_t i = 0; i < gens && st == GA_OK; ++i) st = enqueue_group(gr, i, tables, b);
      if (st == GA_OK)
        st = hip_status(launch_advance(gr.desc, gr.ndesc, gens, b),
                        "advance kernel");
      if (st == GA_OK)
        st = hip_status(hipEventRecord(fork_[gi], b), "hipEventRecord");
      if (st == GA_OK)
        st = hip_status(hipStreamWaitEvent(capture_, fork_[gi], 0),
                        "hipStreamWaitEvent");
    }
    hipError_t ce = hipStreamEndCapture(capture_, &g);
    if (st != GA_OK) return st;
    GA_TRY(ce, "hipStreamEndCapture");
    GA_TRY(hipGraphInstantiate(&graph_, g, nullptr, nullptr, 0),
           "hipGraphInstantiate");
    GA_TRY(hipGraphDestroy(g), "hipGraphDestroy");
    graph_gens_ = gens;
  }
  GA_TRY(hipGraphLaunch(graph_, s), "hipGraphLaunch");
  return GA_OK;
}

// Starts a run in place: state reset, initial population, its fitness.
static ga_status start_run(const ga_config* c, const RunBuffers& b,
                           RunState* st, hipStream_t s) {
  // the selection passes expect zero histograms on entry (and leave them so)
  if (b.sel) GA_TRY(hipMemsetAsync(b.sel, 0, sizeof(SelWork), s), "hipMemsetAsync(selection)");
  // the tile selection: no threshold yet
  if (b.pw) GA_TRY(hipMemsetAsync(b.pw->T, 0xff, sizeof(b.pw->T), s), "hipMemsetAsync(selection)");
  // candidate-list elitism: empty lists (the elites of generation 1 are
  // chosen below, once the initial keys exist)
  if (b.ew)
    GA_TRY(hipMemsetAsync(b.earea, 0, kEliteLists * sizeof(uint32_t), s),
           "hipMemsetAsync(candidate lists)");
  GA_TRY(launch_reset_state(st, s), "state kernel");
  GA_TRY(launch_init(c, b.pop_a, s), "init kernel");
  GA_TRY(launch_fitness(c, b.pop_a, b.keys_a, nullptr, st, s), "fitness kernel");
  if (b.ew) {  // the first generation's elites, from the whole initial population
    const PopDesc d = run_desc(c, b, st);
    GA_TRY(launch_select(d, c->elite, b.sel, 0, nullptr, s, b.ew->src, &b.ew->kstar),
           "selection kernels");
  }
  return GA_OK;
}

ga_status start_runs(const ga_config* cfgs, const RunBuffers* bufs,
                     RunState* states, uint32_t count, hipStream_t s) {
  for (uint32_t i = 0; i < count; ++i) {
    ga_status st = start_run(&cfgs[i], bufs[i], &states[i], s);
    if (st != GA_OK) return st;
  }
  return GA_OK;
}

}  // namespace ga

using namespace ga;

extern "C" ga_status ga_run_batch(const ga_config* cfgs, uint32_t count,
                                  ga_result* outs, void* stream) {
  if (!cfgs || !outs || count == 0) {
    set_error("ga_run_batch needs count > 0 configs and results");
    return GA_EINVAL;
  }
  for (uint32_t i = 0; i < count; ++i) {
    ga_status v = validate(&cfgs[i]);
    if (v != GA_OK) return v;
  }
  // The batch runs on a private stream after the caller's stream is idle
  // (the call is synchronous), so its generation chunks can be graphs.
  GA_TRY(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
  hipStream_t s = nullptr;
  GA_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
  std::vector<RunBuffers> bufs(count);
  RunState* states = nullptr;
  RunState* host = nullptr;
  MultiLaunch ml;
  ga_status rc = GA_OK;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    for (auto& b : bufs) free_run(&b);
    if (states) (void)hipFree(states);
    if (host) (void)hipHostFree(host);
    (void)hipStreamDestroy(s);
  };
  do {
    for (uint32_t i = 0; i < count && rc == GA_OK; ++i)
      rc = alloc_run(&cfgs[i], &bufs[i]);
    if (rc != GA_OK) break;
    rc = hip_status(hipMalloc(&states, count * sizeof(RunState)),
                    "hipMalloc(states)");
    if (rc != GA_OK) break;
    rc = hip_status(hipHostMalloc(&host, count * sizeof(RunState),
                                  hipHostMallocDefault),
                    "hipHostMalloc(states)");
    if (rc != GA_OK) break;
    rc = start_runs(cfgs, bufs.data(), states, count, s);
    if (rc != GA_OK) break;
    std::vector<PopDesc> descs(count);
    uint32_t gmax = 0;
    for (uint32_t i = 0; i < count; ++i) {
      descs[i] = run_desc(&cfgs[i], bufs[i], &states[i]);
      gmax = std::max(gmax, cfgs[i].max_generations);
    }
    rc = ml.set(descs.data(), count, s);
    if (rc != GA_OK) break;
    const uint32_t chunk = std::min<uint32_t>(32, std::max<uint32_t>(gmax, 1));
    uint32_t enq = 0;
    bool all_done = false;
    while (!all_done && enq < gmax) {
      rc = ml.launch_chunk(chunk, s);
      if (rc != GA_OK) break;
      enq += chunk;
      rc = hip_status(hipMemcpyAsync(host, states, count * sizeof(RunState),
                                     hipMemcpyDeviceToHost, s),
                      "hipMemcpyAsync(states)");
      if (rc != GA_OK) break;
      rc = hip_status(hipStreamSynchronize(s), "hipStreamSynchronize");
      if (rc != GA_OK) break;
      all_done = true;
      for (uint32_t i = 0; i < count; ++i)
        all_done &= run_done(host[i], cfgs[i].max_generations,
                             (cfgs[i].flags & GA_STOP_ON_FOUND) != 0);
    }
    if (rc != GA_OK) break;
    rc = ml.finish(s);
    if (rc != GA_OK) break;
    rc = hip_status(hipMemcpyAsync(host, states, count * sizeof(RunState),
                                   hipMemcpyDeviceToHost, s),
                    "hipMemcpyAsync(states)");
    if (rc != GA_OK) break;
    rc = hip_status(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (rc != GA_OK) break;
    for (uint32_t i = 0; i < count && rc == GA_OK; ++i)
      rc = read_result(&cfgs[i], host[i], bufs[i].pop_a, bufs[i].pop_b,
                       &outs[i]);
  } while (0);
  cleanup();
  return rc;
}
