// Continuous-batching scheduler for many solver instances on one GPU (ib_server_* in
// include/ibfsi.h).
//
// Requests are solver handles (created, bodies added, not yet prepared) with a number of
// steps and an arrival time.  The scheduler admits a request once it has arrived, a
// slot is free and its device-memory estimate fits in the budget that the running
// requests leave.  Each slot is a host thread with its own non-blocking HIP stream
// (default priority): it prepares the solver, steps it, keeps its results on the host
// (ib_release) and gives its memory back, so the kernels of the running requests
// overlap on the device and a finished request's slot and memory go to the next one.
// Requests are independent: a result does not depend on what else runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "ib_internal.hpp"
#include "ibfsi.h"

namespace {

struct Request {
  ib_solver* solver = nullptr;
  int32_t nsteps = 0;
  double arrival = 0.0;
  int64_t bytes = 0;
  ib_request_info info{};
};

}  // namespace

struct ib_server {
  int32_t max_active = 1;
  int64_t budget = 0;
  int32_t chunk = 50;
  std::vector<Request> req;
  std::vector<hipStream_t> streams;
  std::mutex mu;
  std::condition_variable cv;
};

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

}  // namespace

extern "C" {

ib_status ib_server_create(int32_t max_active, int64_t hbm_budget_bytes, int32_t chunk_steps,
                           ib_server** out) {
  if (!out || max_active < 1 || max_active > 64 || hbm_budget_bytes <= 0) return IB_ERR_ARG;
  *out = nullptr;
  ib_server* sv = new ib_server();
  sv->max_active = max_active;
  sv->budget = hbm_budget_bytes;
  sv->chunk = chunk_steps > 0 ? chunk_steps : 50;
  for (int k = 0; k < max_active; ++k) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      ib_server_destroy(sv);
      return IB_ERR_HIP;
    }
    sv->streams.push_back(st);
  }
  *out = sv;
  return IB_OK;
}

ib_status ib_server_submit(ib_server* sv, ib_solver* s, int32_t nsteps, double arrival,
                           int64_t* ticket) {
  if (!sv || !s || nsteps < 0 || !ticket) return IB_ERR_ARG;
  Request r;
  r.solver = s;
  r.nsteps = nsteps;
  r.arrival = arrival;
  int64_t resident = 0, peak = 0;
  ib_status st = ib_estimate_bytes(s, &resident, &peak);
  if (st) return st;
  r.bytes = peak;
  if (r.bytes > sv->budget) return IB_ERR_BUDGET;
  r.info.ticket = (int64_t)sv->req.size();
  r.info.status = 1;  // waiting
  r.info.arrival = arrival;
  r.info.bytes = r.bytes;
  *ticket = r.info.ticket;
  sv->req.push_back(r);
  return IB_OK;
}

ib_status ib_server_run(ib_server* sv) {
  if (!sv) return IB_ERR_ARG;
  const int nreq = (int)sv->req.size();
  std::vector<int> order(nreq);
  for (int k = 0; k < nreq; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return sv->req[a].arrival < sv->req[b].arrival; });
  std::deque<int> pending(order.begin(), order.end());
  std::vector<int> slot_busy(sv->max_active, 0);
  std::vector<std::thread> threads(sv->max_active);
  int64_t used = 0;
  int running = 0;
  const Clock::time_point t0 = Clock::now();

  auto worker = [sv, t0](int slot, int idx) {
    Request& r = sv->req[idx];
    ib_status st = ib_set_stream(r.solver, sv->streams[slot]);
    if (!st) st = ib_prepare(r.solver);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      r.info.started = seconds_since(t0);
    }
    int done = 0;
    while (!st && done < r.nsteps) {
      const int k = std::min(sv->chunk, r.nsteps - done);
      st = ib_step(r.solver, k);
      if (!st) done += k;
    }
    if (!st) st = ib_sync(r.solver);
    const ib_status rel = ib_release(r.solver);
    if (!st) st = rel;
    std::lock_guard<std::mutex> lk(sv->mu);
    r.info.steps_done = done;
    r.info.finished = seconds_since(t0);
    r.info.status = st;  // 0 = done, negative = failed
    sv->cv.notify_all();
  };

  std::unique_lock<std::mutex> lk(sv->mu);
  while (!pending.empty() || running > 0) {
    // collect finished slots
    for (int k = 0; k < sv->max_active; ++k) {
      if (slot_busy[k] == 0) continue;
      Request& r = sv->req[slot_busy[k] - 1];
      if (r.info.status == 1 || r.info.status == 2) continue;
      lk.unlock();
      threads[k].join();
      lk.lock();
      used -= r.bytes;
      slot_busy[k] = 0;
      --running;
    }
    // admit what has arrived, in arrival order, while slots and memory allow
    const double now = seconds_since(t0);
    while (!pending.empty()) {
      Request& r = sv->req[pending.front()];
      if (r.arrival > now || running >= sv->max_active || used + r.bytes > sv->budget) break;
      int slot = 0;
      while (slot_busy[slot]) ++slot;
      const int idx = pending.front();
      pending.pop_front();
      slot_busy[slot] = idx + 1;
      used += r.bytes;
      ++running;
      r.info.status = 2;  // running
      r.info.admitted = now;
      threads[slot] = std::thread(worker, slot, idx);
    }
    if (pending.empty() && running == 0) break;
    // wait for a worker to finish or for the next arrival
    double wait = 0.002;
    if (!pending.empty()) {
      const double dt = sv->req[pending.front()].arrival - seconds_since(t0);
      if (dt > 0) wait = std::min(wait, dt);
    }
    sv->cv.wait_for(lk, std::chrono::duration<double>(std::max(wait, 1e-4)));
  }
  return IB_OK;
}

ib_status ib_server_info(ib_server* sv, int64_t ticket, ib_request_info* out) {
  if (!sv || !out || ticket < 0 || ticket >= (int64_t)sv->req.size()) return IB_ERR_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->req[ticket].info;
  return IB_OK;
}

ib_status ib_server_destroy(ib_server* sv) {
  if (!sv) return IB_ERR_ARG;
  auto lk = ib::hip_shared_lock();
  for (auto st : sv->streams) (void)hipStreamDestroy(st);
  delete sv;
  return IB_OK;
}

}  // extern "C"
