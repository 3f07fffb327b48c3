// ga_server.hip -- search server: continuous batching of independent runs.
//
// A worker thread owns one stream on the server's device.  Each tick it
// admits pending requests in arrival order, those whose device memory fits
// the HBM budget (and while a run-state slot is free), starts them, advances
// every active run by a few generations with one children launch per
// generation covering all of them, then retires the runs whose state says
// stop.  A pending request that does not fit is passed over by later ones
// that do, at most kMaxBypass times; after that admission waits for it.
// Runs never share buffers, and every random draw is keyed by the run's own
// seed, so a request's result does not depend on what else is in flight.
// When the worker stops (ga_server_stop, or a device error) every request
// not yet finished fails, and later submissions are refused with the
// worker's terminal status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <queue>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ga_internal.h"

namespace ga {

constexpr uint32_t kServerSlots = 4096;    // runs resident at once
constexpr uint32_t kGensPerTick = 4;       // generations between retire checks
constexpr uint32_t kMaxBypass = 64;        // admissions past a waiting request

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t id = 0;
  ga_config cfg{};
  size_t bytes = 0;
  double t_submit = 0, t_done = 0;
  RunBuffers buf;
  uint32_t slot = 0;
  // the server's admission count when this request was first passed over
  uint64_t passed_at = ~0ull;
  enum { kPending, kActive, kDone } phase = kPending;
  ga_status status = GA_OK;
  std::string error;
  ga_result result{};
};

}  // namespace ga

struct ga_server {
  uint64_t budget = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, std::unique_ptr<ga::Request>> reqs;
  uint64_t next_id = 1;
  uint64_t used = 0;
  uint64_t admissions = 0;  // requests admitted so far
  bool quit = false;
  std::thread worker;
  ga_status start_status = GA_OK;
  std::string start_error;
  bool started = false;
  // set when the worker has stopped: the status later submissions get
  ga_status stop_status = GA_OK;
  std::string stop_error;
  bool stopped = false;
};

namespace ga {

static void finish(ga_server* S, Request* r, ga_status st, const char* err) {
  std::lock_guard<std::mutex> lk(S->mu);
  r->status = st;
  if (err) r->error = err;
  r->t_done = now_s();
  r->phase = Request::kDone;
  S->used -= r->bytes;
  S->cv_done.notify_all();
}

static void worker_main(ga_server* S) {
  hipStream_t stream = nullptr;
  RunState* states = nullptr;
  RunState* host = nullptr;
  ga_status st = hip_status(hipSetDevice(S->device), "hipSetDevice");
  if (st == GA_OK)
    st = hip_status(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking),
                    "hipStreamCreate");
  if (st == GA_OK)
    st = hip_status(hipMalloc(&states, kServerSlots * sizeof(RunState)),
                    "hipMalloc(states)");
  if (st == GA_OK)
    st = hip_status(hipHostMalloc(&host, kServerSlots * sizeof(RunState),
                                  hipHostMallocDefault),
                    "hipHostMalloc(states)");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->start_status = st;
    if (st != GA_OK) S->start_error = ga_last_error();
    S->started = true;
    S->cv_done.notify_all();
  }
  // free run-state slots, lowest first, so that the occupied ones stay
  // packed at the front and each tick copies only that range
  std::priority_queue<uint32_t, std::vector<uint32_t>, std::greater<uint32_t>> free_slots;
  for (uint32_t i = 0; i < kServerSlots; ++i) free_slots.push(i);
  std::vector<Request*> active;
  MultiLaunch ml;
  bool changed = false;
  while (st == GA_OK) {
    std::vector<Request*> admit;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->quit) break;
      // arrival order among the requests that fit; one that does not fit
      // is passed over, up to kMaxBypass times, then waited for
      for (auto it = S->pending.begin();
           it != S->pending.end() && active.size() + admit.size() < kServerSlots;) {
        Request* r = S->reqs[*it].get();
        if (S->used + r->bytes > S->budget) {
          if (r->passed_at == ~0ull) r->passed_at = S->admissions;
          if (S->admissions - r->passed_at >= kMaxBypass) break;
          ++it;
          continue;
        }
        it = S->pending.erase(it);
        S->used += r->bytes;
        ++S->admissions;
        admit.push_back(r);
      }
      if (active.empty() && admit.empty()) {
        S->cv_work.wait_for(lk, std::chrono::milliseconds(20));
        continue;
      }
    }
    for (Request* r : admit) {
      ga_status a = alloc_run(&r->cfg, &r->buf);
      if (a == GA_OK) {
        r->slot = free_slots.top();
        free_slots.pop();
        a = start_runs(&r->cfg, &r->buf, &states[r->slot], 1, stream);
      }
      if (a != GA_OK) {
        free_run(&r->buf);
        finish(S, r, a, ga_last_error());
        continue;
      }
      {
        std::lock_guard<std::mutex> lk(S->mu);
        r->phase = Request::kActive;
      }
      active.push_back(r);
      changed = true;
    }
    if (changed) {
      std::vector<PopDesc> descs;
      for (Request* r : active)
        descs.push_back(run_desc(&r->cfg, r->buf, &states[r->slot]));
      st = ml.set(descs.data(), (uint32_t)descs.size(), stream);
      if (st != GA_OK) break;
      changed = false;
    }
    st = ml.launch_chunk(kGensPerTick, stream);
    if (st != GA_OK) break;
    uint32_t used_slots = 0;
    for (Request* r : active) used_slots = std::max(used_slots, r->slot + 1);
    st = hip_status(hipMemcpyAsync(host, states, used_slots * sizeof(RunState),
                                   hipMemcpyDeviceToHost, stream),
                    "hipMemcpyAsync(states)");
    if (st == GA_OK)
      st = hip_status(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (st != GA_OK) break;
    std::vector<Request*> still;
    for (Request* r : active) {
      if (!run_done(host[r->slot], r->cfg.max_generations,
                    (r->cfg.flags & GA_STOP_ON_FOUND) != 0)) {
        still.push_back(r);
        continue;
      }
      const PopDesc d = run_desc(&r->cfg, r->buf, &states[r->slot]);
      ga_status rr = hip_status(launch_finish_one(d, stream), "finish kernel");
      if (rr == GA_OK)
        rr = hip_status(hipMemcpyAsync(&host[r->slot], &states[r->slot],
                                       sizeof(RunState), hipMemcpyDeviceToHost,
                                       stream),
                        "hipMemcpyAsync(state)");
      if (rr == GA_OK)
        rr = hip_status(hipStreamSynchronize(stream), "hipStreamSynchronize");
      if (rr == GA_OK)
        rr = read_result(&r->cfg, host[r->slot], r->buf.pop_a, r->buf.pop_b,
                         &r->result);
      free_run(&r->buf);
      free_slots.push(r->slot);
      finish(S, r, rr, rr == GA_OK ? nullptr : ga_last_error());
      changed = true;
    }
    active.swap(still);
  }
  // a stop request or a device error ends the worker: everything still
  // queued or running fails with that status, and so does every later
  // submission (recorded in the same critical section that empties the
  // queue, so a submission either lands before it and fails here, or sees
  // the status)
  const ga_status end = st == GA_OK ? GA_ESTOPPED : st;
  const std::string err = st == GA_OK ? "server stopped" : ga_last_error();
  if (stream) (void)hipStreamSynchronize(stream);
  for (Request* r : active) {
    free_run(&r->buf);
    finish(S, r, end, err.c_str());
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (uint64_t id : S->pending) {
      Request* r = S->reqs[id].get();
      r->status = end;
      r->error = err;
      r->t_done = now_s();
      r->phase = Request::kDone;
    }
    S->pending.clear();
    S->stop_status = end;
    S->stop_error = err;
    S->stopped = true;
    S->cv_done.notify_all();
  }
  if (states) (void)hipFree(states);
  if (host) (void)hipHostFree(host);
  if (stream) (void)hipStreamDestroy(stream);
}

static ga_status copy_out(Request* r, ga_result* out) {
  if (r->status != GA_OK) {
    set_error("%s", r->error.c_str());
    return r->status;
  }
  *out = r->result;
  return GA_OK;
}

}  // namespace ga

using namespace ga;

extern "C" {

ga_status ga_server_create(uint64_t hbm_budget_bytes, int device,
                           ga_server** out) {
  if (!out || hbm_budget_bytes == 0) {
    set_error("ga_server_create needs a budget and an output handle");
    return GA_EINVAL;
  }
  ga_server* S = new ga_server();
  S->budget = hbm_budget_bytes;
  S->device = device;
  S->worker = std::thread(worker_main, S);
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&] { return S->started; });
  if (S->start_status != GA_OK) {
    const ga_status st = S->start_status;
    const std::string e = S->start_error;
    lk.unlock();
    S->quit = true;
    S->worker.join();
    delete S;
    set_error("%s", e.c_str());
    return st;
  }
  *out = S;
  return GA_OK;
}

ga_status ga_submit(ga_server* S, const ga_config* cfg, uint64_t* request_id) {
  if (!S || !request_id) {
    set_error("ga_submit needs a server and an id output");
    return GA_EINVAL;
  }
  ga_status v = validate(cfg);
  if (v != GA_OK) return v;
  const size_t bytes = run_bytes(cfg);
  if (bytes > S->budget) {
    set_error("request needs %zu bytes, the budget is %llu", bytes,
              (unsigned long long)S->budget);
    return GA_EBUDGET;
  }
  auto r = std::make_unique<Request>();
  r->cfg = *cfg;
  r->bytes = bytes;
  r->t_submit = now_s();
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stopped) {
    set_error("the server has stopped: %s", S->stop_error.c_str());
    return S->stop_status;
  }
  r->id = S->next_id++;
  *request_id = r->id;
  S->pending.push_back(r->id);
  S->reqs[r->id] = std::move(r);
  S->cv_work.notify_all();
  return GA_OK;
}

ga_status ga_poll(ga_server* S, uint64_t id, ga_result* out) {
  if (!S || !out) {
    set_error("ga_poll needs a server and a result");
    return GA_EINVAL;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) {
    set_error("unknown request %llu", (unsigned long long)id);
    return GA_ENOTFOUND;
  }
  if (it->second->phase != Request::kDone) return GA_PENDING;
  return copy_out(it->second.get(), out);
}

ga_status ga_wait(ga_server* S, uint64_t id, ga_result* out) {
  if (!S || !out) {
    set_error("ga_wait needs a server and a result");
    return GA_EINVAL;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) {
    set_error("unknown request %llu", (unsigned long long)id);
    return GA_ENOTFOUND;
  }
  Request* r = it->second.get();
  S->cv_done.wait(lk, [&] { return r->phase == Request::kDone; });
  return copy_out(r, out);
}

ga_status ga_request_latency(ga_server* S, uint64_t id, double* seconds) {
  if (!S || !seconds) {
    set_error("ga_request_latency needs a server and an output");
    return GA_EINVAL;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) {
    set_error("unknown request %llu", (unsigned long long)id);
    return GA_ENOTFOUND;
  }
  if (it->second->phase != Request::kDone) return GA_PENDING;
  *seconds = it->second->t_done - it->second->t_submit;
  return GA_OK;
}

static void stop_worker(ga_server* S) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->quit = true;
    S->cv_work.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
}

ga_status ga_server_stop(ga_server* S) {
  if (!S) {
    set_error("server is NULL");
    return GA_EINVAL;
  }
  stop_worker(S);
  return GA_OK;
}

ga_status ga_server_destroy(ga_server* S) {
  if (!S) {
    set_error("server is NULL");
    return GA_EINVAL;
  }
  stop_worker(S);
  delete S;
  return GA_OK;
}

}  // extern "C"
