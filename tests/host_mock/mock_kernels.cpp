// CPU stand-ins for libga's launchers: they touch the buffers a kernel would
// read and write (so a sanitizer sees stale or freed buffers) and move the
// run state the way the kernels do.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <set>
#include "ga_internal.h"

namespace ga {
// a small integer mixer for the stand-ins' pseudo-random choices
static uint64_t mix(uint64_t x) {
  x = (x ^ (x >> 31)) * 0x9E3779B97F4A7C15ull;
  return x ^ (x >> 29);
}
static size_t row_words(const PopDesc& d) { return (size_t)d.m * col_words(d.m); }
static void touch_gen(const PopDesc& d, uint32_t G) {
  uint32_t* pop = (G & 1u) ? d.pop_b : d.pop_a;
  uint32_t* keys = (G & 1u) ? d.keys_b : d.keys_a;
  volatile uint32_t x = pop[0] + pop[(size_t)d.n * row_words(d) - 1] + keys[0] + keys[d.n - 1];
  (void)x;
  keys[0] = (uint32_t)(mix(d.seed * 131 + G) & 0xffffff);
  keys[d.n - 1] = 7;
}
static void child_gen(const PopDesc& d, uint32_t node) {
  RunState* st = d.state;
  const uint32_t G = st->gen_base + node + 1;
  if (G > d.max_gen) return;
  if (d.stop_on_found && st->found_gen < G) return;
  touch_gen(d, G - 1);
  touch_gen(d, G);
  if (d.m <= 20 && mix(d.seed * 977 + G) % (d.m * 3) == 0 && G < st->found_gen) st->found_gen = G;
}
hipError_t launch_init(const ga_config* c, uint32_t* pop, hipStream_t s) {
  const size_t w = (size_t)c->n * c->m * col_words(c->m);
  mock_enqueue(s, [=] { pop[0] = 0; pop[w - 1] = 0; });
  return hipSuccess;
}
hipError_t launch_fitness(const ga_config* c, const uint32_t* pop, uint32_t* keys, uint32_t* comps,
                          RunState* st, hipStream_t s) {
  const uint32_t n = c->n;
  mock_enqueue(s, [=] { for (uint32_t i = 0; i < n; ++i) keys[i] = 1000 + (i % 97); volatile uint32_t x = pop[0]; (void)x; (void)comps; (void)st; });
  return hipSuccess;
}
hipError_t launch_fitness_mfma(const ga_config*, const uint32_t*, uint32_t*, uint32_t*, RunState*, uint64_t, uint32_t, hipStream_t) { return hipSuccess; }
hipError_t launch_fitness_repeat(const ga_config*, const uint32_t*, uint32_t*, uint32_t, uint32_t, hipStream_t) { return hipSuccess; }
hipError_t launch_select(const PopDesc&, uint32_t, SelWork*, uint32_t, const uint32_t*, hipStream_t, uint32_t*, uint32_t*) { return hipSuccess; }
hipError_t launch_perm_table(const PopDesc&, uint32_t, uint32_t, uint32_t*, hipStream_t, bool) { return hipSuccess; }
hipError_t launch_elite_select(const PopDesc&, uint32_t, hipStream_t) { return hipSuccess; }
hipError_t launch_elite_select_multi(const PopDesc*, const uint32_t*, uint32_t, uint32_t, hipStream_t) { return hipSuccess; }
hipError_t launch_paper_select(const PopDesc&, uint32_t, uint32_t*, hipStream_t) { return hipSuccess; }
hipError_t launch_paper_select_multi(const PopDesc*, const uint32_t*, uint32_t, uint32_t, hipStream_t) { return hipSuccess; }
hipError_t launch_children(const PopDesc* descs, const uint32_t* map, uint32_t blocks, uint32_t m,
                           uint32_t lanes, uint32_t node, hipStream_t s) {
  mock_enqueue(s, [=] {
    std::set<uint32_t> seen;
    for (uint32_t b = 0; b < blocks; ++b) {
      const uint32_t j = map[b];
      if (seen.insert(j).second) {
        const PopDesc& d = descs[j];
        if (d.m != m || d.lanes != lanes) { fprintf(stderr, "bad group\n"); abort(); }
        if (d.block_begin > b || b - d.block_begin >= d.nblocks) { fprintf(stderr, "bad map\n"); abort(); }
        child_gen(d, node);
      }
    }
  });
  return hipSuccess;
}
hipError_t launch_children_one(const PopDesc& d, uint32_t node, hipStream_t s) {
  const PopDesc dd = d;
  mock_enqueue(s, [=] { child_gen(dd, node); });
  return hipSuccess;
}
hipError_t launch_advance(const PopDesc* descs, uint32_t ndesc, uint32_t k, hipStream_t s) {
  mock_enqueue(s, [=] { for (uint32_t i = 0; i < ndesc; ++i) descs[i].state->gen_base += k; });
  return hipSuccess;
}
hipError_t launch_advance_one(RunState* st, uint32_t k, hipStream_t s) {
  mock_enqueue(s, [=] { st->gen_base += k; });
  return hipSuccess;
}
static void finish_d(const PopDesc& d) {
  RunState* st = d.state;
  const uint32_t g = (d.stop_on_found && st->found_gen <= d.max_gen) ? st->found_gen : d.max_gen;
  const uint32_t* keys = (g & 1u) ? d.keys_b : d.keys_a;
  unsigned long long best = ~0ull;
  for (uint32_t i = 0; i < d.n; ++i) {
    const unsigned long long v = ((unsigned long long)keys[i] << 32) | i;
    if (v < best) best = v;
  }
  if (d.stop_on_found && st->found_gen <= d.max_gen) best = (best & 0xffffffffull);
  st->best = best;
  st->final_gen = g;
}
hipError_t launch_finish(const PopDesc* descs, uint32_t ndesc, hipStream_t s) {
  mock_enqueue(s, [=] { for (uint32_t i = 0; i < ndesc; ++i) finish_d(descs[i]); });
  return hipSuccess;
}
hipError_t launch_finish_one(const PopDesc& d, hipStream_t s) {
  const PopDesc dd = d;
  mock_enqueue(s, [=] { finish_d(dd); });
  return hipSuccess;
}
hipError_t launch_reset_state(RunState* st, hipStream_t s) {
  mock_enqueue(s, [=] { st->best = ~0ull; st->gen_base = 0; st->found_gen = ~0u; st->final_gen = 0; });
  return hipSuccess;
}
hipError_t launch_set_state(RunState* st, uint32_t gen, hipStream_t s) {
  mock_enqueue(s, [=] { st->best = ~0ull; st->gen_base = gen; st->found_gen = ~0u; st->final_gen = gen + 1; });
  return hipSuccess;
}
hipError_t launch_check(const ga_config*, const uint32_t*, uint32_t*, hipStream_t) { return hipSuccess; }
hipError_t launch_pack(const ga_config*, const int8_t*, uint32_t*, uint32_t*, hipStream_t) { return hipSuccess; }
hipError_t launch_unpack(const ga_config*, const uint32_t*, int8_t*, hipStream_t) { return hipSuccess; }
}  // namespace ga
