// Continuous-batching server for RVE crack-length solves on one GPU.
//
// Requests (one RVE problem and a number of crack-length increments each)
// are queued on submission and admitted while a slot is free and their
// device footprint fits into the memory budget that the running requests
// leave.  Each slot is a host thread with its own non-blocking HIP stream
// (default priority): an admitted request is created on that stream,
// bootstrapped and stepped through its increments, so the kernels of the
// requests in flight overlap on the device, and a request submitted while
// others run starts as soon as a slot and memory are free.  Admission is
// first-fit over the queue in arrival order; a request that has been
// overtaken kMaxSkips times blocks further overtaking until it fits.
//
// Batching: the FP32 Krylov solves of the mixed-precision requests (the bulk
// of an increment) go to one engine thread (csrc/batch.hpp) that groups the
// solves in flight by grid and advances each group by a fixed chunk of
// BiCGSTAB iterations per launch sequence, replayed from a captured HIP
// graph: every kernel of a chunk covers all solves of the group, and a solve
// joins or leaves its group at chunk boundaries.  The rest of each
// increment (residual, Newton update, FP64 refinement) runs on the slot's
// stream.
//
// A solve depends only on its own inputs: all reductions are fixed-order per
// RVE and every buffer is written before it is read, so a request gives the
// same results alone and in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "pff.h"

namespace {

constexpr int kMaxSkips = 8;
constexpr int kMaxSlots = 64;

enum { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };

struct Request {
  uint64_t ticket = 0;
  pff_grid grid{};
  std::vector<pff_phase> phases;
  std::vector<uint8_t> pid, mask;
  bool has_mask = false;
  pff_params prm{};
  int n_inc = 0;
  size_t footprint = 0;
  int state = RQ_QUEUED;
  pff_status status = PFF_QUEUED;
  std::string err;
  std::vector<pff_increment_result> results;
  double a0 = 0.0, E_s = 0.0;
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
  int slot = -1;
  int skipped = 0;
  int waiters = 0;        // threads inside pff_server_wait on this request
};

}  // namespace

struct pff_server {
  int device = 0;
  pff_allocator allocator{nullptr, nullptr, nullptr};   // for every request's solver
  pff::KBatcher* kb = nullptr;                           // batched FP32 inner solves (or null)
  size_t budget = 0;
  int nslots = 0;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::map<uint64_t, std::unique_ptr<Request>> all;
  uint64_t next_ticket = 1;
  size_t in_use = 0, peak = 0;
  int running = 0, max_running = 0;
  long long submitted = 0, completed = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0;
  std::string err;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

// First admissible request in arrival order (removed from the queue), or null.
Request* pick(pff_server* S) {
  for (size_t i = 0; i < S->queue.size(); ++i) {
    Request* q = S->queue[i];
    if (q->footprint <= S->budget - S->in_use) {
      for (size_t j = 0; j < i; ++j) S->queue[j]->skipped++;
      S->queue.erase(S->queue.begin() + (long)i);
      return q;
    }
    if (q->skipped >= kMaxSkips) return nullptr;
  }
  return nullptr;
}

// Runs one request on the slot's stream.  Everything the request reports is
// written under the server lock (pff_server_info reads it while it runs).
void run_request(pff_server* S, Request* r, hipStream_t st) {
  pff_solver* s = nullptr;
  pff_status status = pff_create(&r->grid, r->phases.data(), (int)r->phases.size(), r->pid.data(),
                                 r->has_mask ? r->mask.data() : nullptr, &r->prm,
                                 S->allocator.alloc ? &S->allocator : nullptr, st, &s);
  if (status != PFF_OK) {
    std::lock_guard<std::mutex> lk(S->m);
    r->status = status;
    r->err = "pff_create failed";
    return;
  }
  try {
    pff::serving_shapes(s);
    pff::kbatcher_attach(s, S->kb);
  } catch (const std::exception& e) {
    pff_destroy(s);
    std::lock_guard<std::mutex> lk(S->m);
    r->status = PFF_ERR_DEVICE;
    r->err = e.what();
    return;
  }
  double a0 = 0.0, E_s = 0.0;
  status = pff_bootstrap(s, &a0, &E_s);
  {
    std::lock_guard<std::mutex> lk(S->m);
    r->a0 = a0;
    r->E_s = E_s;
  }
  if (status == PFF_OK) {
    for (int k = 0; k < r->n_inc; ++k) {
      pff_increment_result res;
      std::memset(&res, 0, sizeof(res));
      const pff_status st2 = pff_step(s, &res);
      {
        std::lock_guard<std::mutex> lk(S->m);
        r->results.push_back(res);
      }
      if (st2 != PFF_OK) {
        status = st2;
        break;
      }
    }
  }
  std::string err;
  if (status != PFF_OK) {
    const char* e = pff_last_error(s);
    err = e ? e : "";
  }
  pff_destroy(s);
  std::lock_guard<std::mutex> lk(S->m);
  r->err = err;
  r->status = status;
  if (status != PFF_OK)
    S->err = "request " + std::to_string(r->ticket) + " (status " + std::to_string(status) + "): " + err;
}

void worker(pff_server* S, int slot) {
  (void)hipSetDevice(S->device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->m);
      S->cv_work.wait(lk, [&] { return S->stop || (r = pick(S)) != nullptr; });
      if (!r) break;
      r->state = RQ_RUNNING;
      r->slot = slot;
      r->t_admit = S->now();
      S->in_use += r->footprint;
      S->peak = std::max(S->peak, S->in_use);
      S->running++;
      S->max_running = std::max(S->max_running, S->running);
    }
    if (have_stream) run_request(S, r, st);
    {
      std::lock_guard<std::mutex> lk(S->m);
      if (!have_stream) {
        r->status = PFF_ERR_DEVICE;
        r->err = "could not create a stream for the slot";
      }
      S->in_use -= r->footprint;
      S->running--;
      S->completed++;
      r->t_done = S->now();
      r->state = RQ_DONE;
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  if (have_stream) (void)hipStreamDestroy(st);
}

Request* find(pff_server* S, uint64_t ticket) {
  auto it = S->all.find(ticket);
  return it == S->all.end() ? nullptr : it->second.get();
}

}  // namespace

extern "C" {

pff_status pff_server_create(size_t hbm_budget_bytes, int max_slots, const pff_allocator* allocator,
                             pff_server** out) {
  if (!out) return PFF_ERR_ARG;
  *out = nullptr;
  if (hbm_budget_bytes == 0 || max_slots < 1 || max_slots > kMaxSlots) return PFF_ERR_ARG;
  if (allocator && ((allocator->alloc == nullptr) != (allocator->free == nullptr))) return PFF_ERR_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return PFF_ERR_DEVICE;
  auto* S = new (std::nothrow) pff_server();
  if (!S) return PFF_ERR_OOM;
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return PFF_ERR_DEVICE;
  }
  S->budget = hbm_budget_bytes;
  S->nslots = max_slots;
  if (allocator && allocator->alloc) S->allocator = *allocator;
  {
    auto envi = [](const char* k, int d) {
      const char* v = std::getenv(k);
      return v ? std::atoi(v) : d;
    };
    if (envi("PFF_SERVER_BATCH", 1) != 0) {
      S->kb = pff::kbatcher_create(S->device, envi("PFF_BATCH_MAX", 8), envi("PFF_BATCH_CHUNK", 4),
                                   envi("PFF_BATCH_GRAPH", 1));
      if (!S->kb) {
        delete S;
        return PFF_ERR_OOM;
      }
    }
  }
  S->t0 = std::chrono::steady_clock::now();
  for (int k = 0; k < max_slots; ++k) S->workers.emplace_back(worker, S, k);
  *out = S;
  return PFF_OK;
}

pff_status pff_server_submit(pff_server* S, const pff_grid* grid, const pff_phase* phases, int n_phases,
                             const uint8_t* phase_id, const uint8_t* crack_mask, const pff_params* params,
                             int n_increments, uint64_t* ticket) {
  if (!S || !grid || !phases || n_phases < 1 || !phase_id || !params || n_increments < 1 || !ticket)
    return PFF_ERR_ARG;
  size_t fp = 0;
  if (pff_footprint_bytes(grid, params->precision, &fp) != PFF_OK) return PFF_ERR_ARG;
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return PFF_ERR_OOM;
  const size_t N = (size_t)grid->nx * grid->ny * grid->nz;
  r->grid = *grid;
  r->phases.assign(phases, phases + n_phases);
  r->pid.assign(phase_id, phase_id + N);
  if (crack_mask) {
    r->mask.assign(crack_mask, crack_mask + N);
    r->has_mask = true;
  }
  r->prm = *params;
  r->n_inc = n_increments;
  r->footprint = fp;
  {
    std::lock_guard<std::mutex> lk(S->m);
    if (fp > S->budget) {
      S->err = "request footprint exceeds the server memory budget";
      return PFF_ERR_ARG;
    }
    if (S->stop) {
      S->err = "server is shutting down";
      return PFF_ERR_STATE;
    }
    r->ticket = S->next_ticket++;
    r->t_submit = S->now();
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->all[r->ticket] = std::move(r);
    S->submitted++;
  }
  S->cv_work.notify_all();
  return PFF_OK;
}

pff_status pff_server_wait(pff_server* S, uint64_t ticket, double timeout_seconds) {
  if (!S) return PFF_ERR_ARG;
  std::unique_lock<std::mutex> lk(S->m);
  Request* r = find(S, ticket);
  if (!r) return PFF_ERR_ARG;
  // the request stays alive while it has waiters: pff_server_release refuses it
  r->waiters++;
  auto done = [&] { return r->state == RQ_DONE; };
  if (timeout_seconds < 0) {
    S->cv_done.wait(lk, done);
  } else {
    S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_seconds), done);
  }
  r->waiters--;
  return done() ? PFF_OK : PFF_QUEUED;
}

pff_status pff_server_info(pff_server* S, uint64_t ticket, pff_request_info* out) {
  if (!S || !out) return PFF_ERR_ARG;
  std::lock_guard<std::mutex> lk(S->m);
  Request* r = find(S, ticket);
  if (!r) return PFF_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  out->ticket = r->ticket;
  out->state = r->state;
  out->status = r->status;
  out->n_done = (int)r->results.size();
  out->slot = r->slot;
  out->footprint = r->footprint;
  out->t_submit = r->t_submit;
  out->t_admit = r->t_admit;
  out->t_done = r->t_done;
  out->a0 = r->a0;
  out->E_s = r->E_s;
  return PFF_OK;
}

pff_status pff_server_results(pff_server* S, uint64_t ticket, pff_increment_result* out, int capacity,
                              int* n_out) {
  if (!S || !n_out || capacity < 0 || (capacity > 0 && !out)) return PFF_ERR_ARG;
  std::lock_guard<std::mutex> lk(S->m);
  Request* r = find(S, ticket);
  if (!r) return PFF_ERR_ARG;
  if (r->state != RQ_DONE) return PFF_QUEUED;
  const int n = std::min<int>(capacity, (int)r->results.size());
  for (int k = 0; k < n; ++k) out[k] = r->results[k];
  *n_out = (int)r->results.size();
  return PFF_OK;
}

pff_status pff_server_release(pff_server* S, uint64_t ticket) {
  if (!S) return PFF_ERR_ARG;
  std::lock_guard<std::mutex> lk(S->m);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return PFF_ERR_ARG;
  if (it->second->state != RQ_DONE || it->second->waiters > 0) return PFF_ERR_STATE;
  S->all.erase(it);
  return PFF_OK;
}

pff_status pff_server_get_stats(pff_server* S, pff_server_stats* out) {
  if (!S || !out) return PFF_ERR_ARG;
  std::lock_guard<std::mutex> lk(S->m);
  std::memset(out, 0, sizeof(*out));
  out->submitted = S->submitted;
  out->completed = S->completed;
  out->queued = (long long)S->queue.size();
  out->running = S->running;
  out->max_running = S->max_running;
  out->slots = S->nslots;
  out->budget = S->budget;
  out->bytes_in_use = S->in_use;
  out->peak_bytes = S->peak;
  out->clock = S->now();
  if (S->kb) {
    pff::KBatcherStats b;
    pff::kbatcher_stats(S->kb, &b);
    out->batch_chunks = b.chunks;
    out->batch_solves = b.solves;
    out->batch_iterations = b.iterations;
    out->batch_graphs = b.graphs;
    out->batch_max = b.max_batch;
    out->batch_mean = b.chunks > 0 ? double(b.rve_chunks) / double(b.chunks) : 0.0;
  }
  return PFF_OK;
}

const char* pff_server_last_error(pff_server* S) { return S ? S->err.c_str() : "null server"; }

void pff_server_destroy(pff_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->m);
    S->stop = true;
    for (Request* q : S->queue) {
      q->status = PFF_ERR_STATE;
      q->err = "server shut down before the request was admitted";
      q->state = RQ_DONE;
    }
    S->queue.clear();
  }
  S->cv_work.notify_all();
  S->cv_done.notify_all();
  for (auto& t : S->workers) t.join();
  pff::kbatcher_destroy(S->kb);
  delete S;
}

}  // extern "C"
