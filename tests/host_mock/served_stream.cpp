// Streams requests into the server as the served workload does (arrivals
// spread over time, runs admitted and retired while others run) on the CPU
// stand-in of the HIP runtime.  Arguments: requests, microseconds between
// submissions, largest population.  Prints "all done" when every request
// has finished.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>
#include "ga.h"

int main(int argc, char** argv) {
  const int count = argc > 1 ? atoi(argv[1]) : 2000;
  const int gap_us = argc > 2 ? atoi(argv[2]) : 500;
  const int maxn = argc > 3 ? atoi(argv[3]) : 5000;
  ga_server* S = nullptr;
  if (ga_server_create(200ull * 1000 * 1000 * 1000, 0, &S) != GA_OK) { printf("create failed: %s\n", ga_last_error()); return 1; }
  std::mt19937_64 rng(5);
  std::vector<uint64_t> ids;
  for (int i = 0; i < count; ++i) {
    ga_config c;
    memset(&c, 0, sizeof c);
    c.m = 4 * (2 + rng() % 15);
    c.n = 1000 + rng() % (maxn - 999);
    c.seed = 5000000 + i;
    c.max_generations = 200 + rng() % 200;
    c.fitness = GA_FIT_SQ;
    c.selection = GA_SEL_TOURNAMENT;
    c.tournament_k = 2;
    c.xo_threshold = 1ull << 31;
    c.mut_threshold = 429496730;
    c.nc = 1;
    c.nr = 1;
    c.flags = GA_STOP_ON_FOUND;
    uint64_t id;
    ga_status st = ga_submit(S, &c, &id);
    if (st != GA_OK) { printf("submit %d failed: %s\n", i, ga_last_error()); return 1; }
    ids.push_back(id);
    std::this_thread::sleep_for(std::chrono::microseconds(gap_us));
    if ((i + 1) % 500 == 0) printf("submitted %d\n", i + 1), fflush(stdout);
  }
  static ga_result r;
  int found = 0;
  for (uint64_t id : ids) {
    ga_status st = ga_wait(S, id, &r);
    if (st != GA_OK) { printf("wait failed: %s\n", ga_last_error()); return 1; }
    found += r.found;
  }
  printf("all done, found %d\n", found);
  ga_server_destroy(S);
  return 0;
}
