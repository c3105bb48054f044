// Serving: continuous batching of forward and adjoint matvec requests against
// device-resident operators, with workspace admission by a device-memory
// budget.
//
// A worker thread owns n_slots HIP streams.  Requests wait in one FIFO queue;
// whenever a slot is free the worker takes the oldest request plus every
// later queued request for the same operator and direction (up to
// max_batch_rhs right-hand sides in total) and launches them as one
// multi-right-hand-side matvec, provided its workspace fits in what is left
// of the budget.  Batches on different slots run concurrently on the device.
// Each batch ends with an event on its slot's stream; while any batch runs,
// the worker polls those events (a stream host callback would add ~35 us to
// every batch on this runtime), marks a finished batch complete and records
// each request's latency (submit to completion, steady clock).  The worker
// therefore keeps one CPU core busy while the device has work from it.
// Requests that arrive while others run are admitted as soon as a slot and
// workspace free up: nothing waits for a batch to fill.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ftm.h"
#include "ftm_arena.h"
#include "ftm_runtime.h"

using ftm_rt::Arena;
using ftm_rt::fail;
using ftm_rt::fail_hip;

namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

// Before blocking on a condition variable, the worker (idle) and a waiter
// spin this long on a counter: a futex wake-up costs ~10 us, which is a
// sizeable part of a small request's latency.
constexpr double kSpinSeconds = 100e-6;

// Spin until counter moves away from seen or the spin time is up.
void spin_on(const std::atomic<uint64_t>& counter, uint64_t seen) {
  const double t0 = now_s();
  while (counter.load(std::memory_order_acquire) == seen && now_s() - t0 < kSpinSeconds) std::this_thread::yield();
}

struct Request {
  uint64_t ticket;
  ftm_operator op;
  bool adjoint;
  const double* x;
  double* y;
  int64_t nrhs;
  double t_submit;
  hipEvent_t ready;  // optional: x is valid once this event has completed
};

enum : uint8_t { ST_QUEUED = 1, ST_RUNNING = 2, ST_DONE = 3, ST_FAILED = 4 };

}  // namespace

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;  // recorded after the batch's last kernel
  bool busy = false;          // slots are touched by the worker thread only
  std::vector<Request> reqs;
  ftm_rt::Exec ex;  // the batch's configuration, copied when it was admitted
  size_t ws_off = 0, ws_bytes = 0;
  int64_t nrhs = 0;
  const double** h_ptrs = nullptr;  // pinned: [max_rhs] inputs then [max_rhs] outputs
  void* d_ptrs = nullptr;
};

struct ftm_server_s {
  int device = 0;
  void* arena_base = nullptr;
  size_t budget = 0;
  Arena arena;
  int64_t max_batch_rhs = 1;
  std::vector<Slot> slots;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> queue;
  std::vector<double> latency;  // by ticket - 1
  std::vector<uint8_t> state;
  uint64_t next_ticket = 1;
  std::atomic<uint64_t> n_submitted{0}, n_finished{0};  // spin targets; mu guards the rest
  bool stop = false;
  bool budget_blocked = false;  // the queue head waits for workspace to free up
  std::string error;
  std::thread worker;

  ftm_server_stats stats{};
  int64_t inflight_requests = 0;

  void run();
  void launch(Slot& s, std::vector<Request>&& batch, const ftm_rt::Exec& ex, size_t off, size_t bytes,
              int64_t nrhs);
  void fail_head(const std::string& why);
  void finish(Slot& s, hipError_t q, double t);
};

// A slot's batch has ended (its event completed at time t, or the query
// failed with q): stamp or fail its requests and free the slot (lock held).
void ftm_server_s::finish(Slot& s, hipError_t q, double t) {
  if (q == hipSuccess) {
    for (const Request& r : s.reqs) {
      latency[r.ticket - 1] = t - r.t_submit;
      state[r.ticket - 1] = ST_DONE;
    }
    stats.completed += s.reqs.size();
  } else {
    error = std::string("serving batch: ") + hipGetErrorString(q);
    for (const Request& r : s.reqs) state[r.ticket - 1] = ST_FAILED;
    stats.failed += s.reqs.size();
  }
  arena.release(s.ws_off, s.ws_bytes);
  inflight_requests -= (int64_t)s.reqs.size();
  s.reqs.clear();
  s.busy = false;
  budget_blocked = false;
  n_finished.fetch_add(1, std::memory_order_release);
  cv_done.notify_all();
}

void ftm_server_s::launch(Slot& s, std::vector<Request>&& batch, const ftm_rt::Exec& ex, size_t off, size_t bytes,
                          int64_t nrhs) {
  s.busy = true;
  s.reqs = std::move(batch);
  s.ex = ex;
  s.ws_off = off;
  s.ws_bytes = bytes;
  s.nrhs = nrhs;
  const ftm_operator op = s.reqs.front().op;
  const bool adj = s.reqs.front().adjoint;
  const int64_t nin = op->Nt * (adj ? op->Nd : op->Nm), nout = op->Nt * (adj ? op->Nm : op->Nd);
  int64_t i = 0;
  for (const Request& r : s.reqs)
    for (int64_t j = 0; j < r.nrhs; ++j, ++i) {
      s.h_ptrs[i] = r.x + j * nin;
      s.h_ptrs[max_batch_rhs + i] = r.y + j * nout;
    }
  for (Request& r : s.reqs) state[r.ticket - 1] = ST_RUNNING;
  stats.batches += 1;
  stats.rhs_launched += (uint64_t)nrhs;
  if ((int64_t)s.reqs.size() > 1) stats.coalesced_requests += s.reqs.size();
  const size_t used = arena.used();
  if (used > stats.peak_workspace_bytes) stats.peak_workspace_bytes = used;

  // enqueue without holding the lock: HIP calls can take a while
  mu.unlock();
  ftm_status st = FTM_OK;
  hipError_t e = hipSuccess;
  for (const Request& r : s.reqs)
    if (r.ready && e == hipSuccess) e = hipStreamWaitEvent(s.stream, r.ready, 0);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s.d_ptrs, s.h_ptrs, 2 * max_batch_rhs * sizeof(void*), hipMemcpyHostToDevice,
                                s.stream);
  if (e == hipSuccess) {
    ftm_rt::MatvecIO io;
    io.xptr = reinterpret_cast<const double* const*>(s.d_ptrs);
    io.yptr = reinterpret_cast<double* const*>(s.d_ptrs) + max_batch_rhs;
    const ftm_rt::Workspace ws =
        ftm_rt::carve_workspace(op, reinterpret_cast<char*>(arena_base) + off, nrhs, adj, s.ex.p);
    st = ftm_rt::run_matvec(op, adj, s.ex, io, nrhs, ws, s.stream);
    if (st == FTM_OK) e = hipEventRecord(s.done, s.stream);
  }
  mu.lock();
  if (e != hipSuccess || st != FTM_OK) {
    error = e != hipSuccess ? std::string("serving launch: ") + hipGetErrorString(e) : std::string(ftm_last_error());
    for (const Request& r : s.reqs) state[r.ticket - 1] = ST_FAILED;
    // nothing was queued after the failing call: wait for what was, then free
    (void)hipStreamSynchronize(s.stream);
    arena.release(s.ws_off, s.ws_bytes);
    inflight_requests -= (int64_t)s.reqs.size();
    stats.failed += s.reqs.size();
    s.reqs.clear();
    s.busy = false;
    cv_done.notify_all();
  }
}

// Fail the queue head (the lock is held).
void ftm_server_s::fail_head(const std::string& why) {
  const Request& head = queue.front();
  error = why;
  state[head.ticket - 1] = ST_FAILED;
  stats.failed += 1;
  inflight_requests -= 1;
  queue.pop_front();
  cv_done.notify_all();
}

void ftm_server_s::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  std::vector<hipError_t> q(slots.size());
  std::vector<double> t_done(slots.size());
  for (;;) {
    // admit: oldest request first, coalescing same-operator same-direction requests
    while (!queue.empty()) {
      Slot* free_slot = nullptr;
      bool any_busy = false;
      for (auto& s : slots) {
        if (!s.busy && !free_slot) free_slot = &s;
        any_busy = any_busy || s.busy;
      }
      if (!free_slot) break;
      const Request head = queue.front();
      // the batch runs the configuration its operator has now
      const ftm_rt::Exec ex0 = head.op->exec(head.adjoint, head.nrhs, false);
      if (Arena::need(head.op->workspace_bytes(head.nrhs, head.adjoint, ex0.p)) > arena.capacity()) {
        // the operator's precision changed after submit to one whose
        // workspace exceeds the whole budget: this request can never run
        fail_head("request needs more workspace than the whole budget at the operator's current precision");
        continue;
      }
      std::vector<size_t> take{0};
      int64_t total = head.nrhs;
      for (size_t i = 1; i < queue.size() && total < max_batch_rhs; ++i) {
        const Request& r = queue[i];
        if (r.op == head.op && r.adjoint == head.adjoint && total + r.nrhs <= max_batch_rhs) {
          take.push_back(i);
          total += r.nrhs;
        }
      }
      ftm_rt::Exec ex = head.op->exec(head.adjoint, total, false);
      size_t off = 0, bytes = head.op->workspace_bytes(total, head.adjoint, ex.p);
      while (!arena.alloc(bytes, &off)) {
        // shrink the batch from the back until it fits; the head alone may
        // have to wait for running batches to release workspace
        if (take.size() == 1) {
          bytes = 0;
          break;
        }
        total -= queue[take.back()].nrhs;
        take.pop_back();
        ex = head.op->exec(head.adjoint, total, false);
        bytes = head.op->workspace_bytes(total, head.adjoint, ex.p);
      }
      if (bytes == 0) {
        if (!any_busy) {
          // cannot happen (the head fits an empty arena), but never wait for a
          // release that no running batch will make
          fail_head("request does not fit the empty workspace arena");
          continue;
        }
        stats.budget_waits += 1;
        budget_blocked = true;
        break;
      }
      std::vector<Request> batch;
      batch.reserve(take.size());
      for (size_t t : take) batch.push_back(queue[t]);
      for (size_t t = take.size(); t-- > 0;) queue.erase(queue.begin() + (std::ptrdiff_t)take[t]);
      launch(*free_slot, std::move(batch), ex, off, bytes, total);
    }

    bool busy = false;
    for (auto& s : slots) busy = busy || s.busy;
    if (stop && queue.empty() && !busy) break;
    if (busy) {
      // poll the running batches' events without the lock (submitters and
      // waiters take it meanwhile), then reap the finished ones
      lk.unlock();
      std::this_thread::yield();
      bool any_done = false;
      for (size_t i = 0; i < slots.size(); ++i) {
        q[i] = slots[i].busy ? hipEventQuery(slots[i].done) : hipErrorNotReady;
        t_done[i] = now_s();
        any_done = any_done || q[i] != hipErrorNotReady;
      }
      lk.lock();
      if (any_done)
        for (size_t i = 0; i < slots.size(); ++i)
          if (q[i] != hipErrorNotReady) finish(slots[i], q[i], t_done[i]);
      continue;
    }
    // nothing runs: spin briefly for a new request, then sleep until there is
    // queued work that is not blocked on the budget, or until a stop
    if (queue.empty() && !stop) {
      const uint64_t seen = n_submitted.load(std::memory_order_acquire);
      lk.unlock();
      spin_on(n_submitted, seen);
      lk.lock();
    }
    cv_work.wait(lk, [&] { return stop || (!queue.empty() && !budget_blocked); });
  }
}

extern "C" {

ftm_status ftm_server_create(ftm_server* out, size_t workspace_budget, int32_t n_slots, int64_t max_batch_rhs) {
  try {
    if (!out) return fail(FTM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (workspace_budget < 4096) return fail(FTM_ERR_INVALID, "workspace budget below 4 KiB");
    if (n_slots < 1 || n_slots > 16) return fail(FTM_ERR_INVALID, "n_slots must be in [1, 16]");
    if (max_batch_rhs < 1 || max_batch_rhs > 4096) return fail(FTM_ERR_INVALID, "max_batch_rhs must be in [1, 4096]");
    ftm_server s0 = new ftm_server_s();
    std::unique_ptr<ftm_server_s> s(s0);
    if (hipGetDevice(&s->device) != hipSuccess) return fail(FTM_ERR_HIP, "hipGetDevice failed");
    s->budget = workspace_budget;
    s->max_batch_rhs = max_batch_rhs;
    if (hipMalloc(&s->arena_base, workspace_budget) != hipSuccess) {
      (void)hipGetLastError();
      return fail(FTM_ERR_OOM, "could not allocate the serving workspace");
    }
    s->arena.reset(workspace_budget);
    s->slots.resize(n_slots);
    auto cleanup = [&](ftm_status st) {
      for (auto& sl : s->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.h_ptrs) (void)hipHostFree(sl.h_ptrs);
        if (sl.d_ptrs) (void)hipFree(sl.d_ptrs);
      }
      (void)hipFree(s->arena_base);
      return st;
    };
    for (int i = 0; i < n_slots; ++i) {
      Slot& sl = s->slots[i];
      if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
        return cleanup(fail(FTM_ERR_HIP, "hipStreamCreateWithFlags failed"));
      if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
        return cleanup(fail(FTM_ERR_HIP, "hipEventCreateWithFlags failed"));
      const size_t pbytes = 2 * (size_t)max_batch_rhs * sizeof(void*);
      if (hipHostMalloc(reinterpret_cast<void**>(&sl.h_ptrs), pbytes, hipHostMallocDefault) != hipSuccess ||
          hipMalloc(&sl.d_ptrs, pbytes) != hipSuccess)
        return cleanup(fail(FTM_ERR_OOM, "pointer-array allocation failed"));
    }
    s->worker = std::thread([p = s.get()] { p->run(); });
    *out = s.release();
    return FTM_OK;
  } catch (...) {
    return fail(FTM_ERR_INVALID, "unexpected exception in ftm_server_create");
  }
}

ftm_status ftm_server_submit(ftm_server s, ftm_operator op, int32_t adjoint, const double* x, double* y,
                             int64_t nrhs, void* ready_event, uint64_t* ticket) {
  if (!s || !op || !x || !y || !ticket) return fail(FTM_ERR_INVALID, "NULL argument");
  if (nrhs < 1 || nrhs > s->max_batch_rhs)
    return fail(FTM_ERR_INVALID, "nrhs must be in [1, max_batch_rhs=" + std::to_string(s->max_batch_rhs) + "]");
  if (op->device != s->device) return fail(FTM_ERR_INVALID, "operator lives on another device");
  const ftm_rt::Exec ex = op->exec(adjoint != 0, nrhs, false);
  if (!op->spec[ex.p.gemv].p) return fail(FTM_ERR_STATE, "spectrum for the configured precision is missing");
  const size_t need = Arena::need(op->workspace_bytes(nrhs, adjoint != 0, ex.p));
  if (need > s->arena.capacity())
    return fail(FTM_ERR_BUDGET, "request needs " + std::to_string(need) +
                                    " workspace bytes, more than the whole budget");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(FTM_ERR_STATE, "server is shutting down");
    Request r{s->next_ticket++, op, adjoint != 0, x, y, nrhs, now_s(), reinterpret_cast<hipEvent_t>(ready_event)};
    s->latency.push_back(NAN);
    s->state.push_back(ST_QUEUED);
    s->queue.push_back(r);
    s->stats.submitted += 1;
    s->inflight_requests += 1;
    if (s->inflight_requests > s->stats.max_inflight_requests) s->stats.max_inflight_requests = s->inflight_requests;
    *ticket = r.ticket;
    s->n_submitted.fetch_add(1, std::memory_order_release);
  }
  s->cv_work.notify_one();
  return FTM_OK;
}

ftm_status ftm_server_poll(ftm_server s, uint64_t ticket, int32_t* done, double* latency_s) {
  if (!s || !done) return fail(FTM_ERR_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket < 1 || ticket >= s->next_ticket) return fail(FTM_ERR_INVALID, "unknown ticket");
  const uint8_t st = s->state[ticket - 1];
  if (st == ST_FAILED) return fail(FTM_ERR_HIP, "request failed: " + s->error);
  *done = st == ST_DONE;
  if (latency_s) *latency_s = s->latency[ticket - 1];
  return FTM_OK;
}

ftm_status ftm_server_wait(ftm_server s, uint64_t ticket, double* latency_s, double timeout_s) {
  if (!s) return fail(FTM_ERR_INVALID, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket < 1 || ticket >= s->next_ticket) return fail(FTM_ERR_INVALID, "unknown ticket");
  auto ready = [&] { return s->state[ticket - 1] >= ST_DONE; };
  // spin while batches keep finishing, for up to the spin time, then block
  for (const double t0 = now_s(); !ready() && now_s() - t0 < kSpinSeconds;) {
    const uint64_t seen = s->n_finished.load(std::memory_order_acquire);
    lk.unlock();
    spin_on(s->n_finished, seen);
    lk.lock();
  }
  if (timeout_s > 0) {
    if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready))
      return fail(FTM_ERR_STATE, "timed out waiting for the request");
  } else {
    s->cv_done.wait(lk, ready);
  }
  if (s->state[ticket - 1] == ST_FAILED) return fail(FTM_ERR_HIP, "request failed: " + s->error);
  if (latency_s) *latency_s = s->latency[ticket - 1];
  return FTM_OK;
}

ftm_status ftm_server_latencies(ftm_server s, uint64_t first_ticket, int64_t n, double* out) {
  if (!s || !out || n < 0) return fail(FTM_ERR_INVALID, "bad argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (first_ticket < 1 || first_ticket + (uint64_t)n > s->next_ticket) return fail(FTM_ERR_INVALID, "tickets out of range");
  for (int64_t i = 0; i < n; ++i) out[i] = s->latency[first_ticket - 1 + i];
  return FTM_OK;
}

ftm_status ftm_server_get_stats(ftm_server s, ftm_server_stats* out) {
  if (!s || !out) return fail(FTM_ERR_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->workspace_in_use_bytes = s->arena.used();
  out->queued_requests = (int64_t)s->queue.size();
  return FTM_OK;
}

ftm_status ftm_server_destroy(ftm_server s) {
  if (!s) return FTM_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();  // drains the queue and every running batch
  ftm_rt::DeviceGuard g(s->device);
  for (auto& sl : s->slots) {
    if (sl.stream) {
      (void)hipStreamSynchronize(sl.stream);
      (void)hipStreamDestroy(sl.stream);
    }
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.h_ptrs) (void)hipHostFree(sl.h_ptrs);
    if (sl.d_ptrs) (void)hipFree(sl.d_ptrs);
  }
  (void)hipFree(s->arena_base);
  delete s;
  return FTM_OK;
}

}  // extern "C"
