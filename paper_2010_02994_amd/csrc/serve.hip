// Continuous-batching server for Hawkes log-likelihood + gradient requests.
//
// Many HMC chains over datasets of uneven size submit one evaluation each per
// leapfrog step.  Dataset times stay resident on the device after
// registration; each request brings its latent locations (device memory owned
// by the client) and its parameters.  A scheduler thread admits requests in
// arrival order while a slot is free and the request's workspace fits in the
// server's HBM arena, groups admitted requests of the same (D, precision)
// into a batch, and launches the batch as one kernel launch per phase on one
// of several streams.  Batches on different streams overlap on the device,
// and requests that arrive while batches run are admitted as soon as slots and
// memory free up.  Each request's work decomposition depends only on its own
// (N, D, precision), so its result is bitwise the same alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hawkes.h"
#include "hawkes_common.hpp"
#include "hawkes_internal.hpp"

namespace hawkes {
namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, capacity) with coalescing of free neighbours.
class Arena {
 public:
  explicit Arena(size_t cap = 0) { reset(cap); }
  void reset(size_t cap) {
    free_.clear();
    if (cap) free_[0] = cap;
    cap_ = cap;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t free_bytes() const {
    size_t s = 0;
    for (auto& kv : free_) s += kv.second;
    return s;
  }
  size_t capacity() const { return cap_; }

 private:
  std::map<size_t, size_t> free_;
  size_t cap_ = 0;
};

struct Dataset {
  double* t = nullptr;   // resident copy (device)
  int64_t n = 0;
  int d = 0;
};

struct Request {
  uint64_t ticket = 0;
  int32_t ds = -1;
  const double* x = nullptr;
  hawkes_params_t p{};
  int prec = 0;
  double* grad_x = nullptr;
  size_t foot = 0, off = 0;
  bool admitted = false, done = false;
  hawkes_result_t res{};
};

struct Batch {
  bool busy = false;
  int nreq = 0;
  std::vector<Request*> reqs;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  ReqDesc* dev_desc = nullptr;    // device copy of the descriptors
  ReqDesc* host_desc = nullptr;   // pinned staging
  double* dev_out = nullptr;      // nreq x 8 results
  double* host_out = nullptr;     // pinned
  uint64_t sim_done_ns = 0;       // simulate mode: virtual completion time
};

}  // namespace
}  // namespace hawkes

struct hawkes_server {
  size_t budget = 0;
  int max_slots = 0;
  bool simulate = false;
  hawkes_allocator_t alloc{};     // device memory source (alloc.alloc == NULL: hipMalloc)
  char* arena_base = nullptr;
  hawkes::Arena arena;
  std::vector<hawkes::Dataset> datasets;
  std::deque<hawkes::Request*> pending;
  std::unordered_map<uint64_t, hawkes::Request*> by_ticket;
  std::vector<hawkes::Batch> batches;
  int active = 0;                 // admitted and not yet completed
  uint64_t next_ticket = 1;
  bool stop = false;
  uint64_t n_batches = 0, n_requests = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
};

namespace hawkes {
namespace {

// Device memory of the server: the caller's allocator when given, else hipMalloc.
// Buffers must come back aligned to 256 bytes.
void* dev_alloc(hawkes_server* S, size_t bytes) {
  void* p = nullptr;
  if (S->alloc.alloc) {
    p = S->alloc.alloc(bytes, S->alloc.ctx);
    if (p && (reinterpret_cast<uintptr_t>(p) & 255u) != 0) {
      S->alloc.free(p, S->alloc.ctx);
      p = nullptr;
    }
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  return p;
}

void dev_free(hawkes_server* S, void* p) {
  if (!p) return;
  if (S->alloc.alloc) S->alloc.free(p, S->alloc.ctx);
  else (void)hipFree(p);
}

size_t footprint(int64_t n, int d, int prec) {
  const size_t ws = hawkes_workspace_bytes(n, d, prec);
  return ws ? (ws + 4095) & ~size_t(4095) : 0;
}

void finish(hawkes_server* S, Request* r, int status, const double* out8) {
  r->res.status = status;
  if (out8) {
    r->res.loglik = out8[0];
    for (int k = 0; k < 6; ++k) r->res.grad_params[k] = out8[1 + k];
  }
  r->res.t_done_ns = now_ns();
  r->done = true;
  if (r->admitted) {
    S->arena.release(r->off, r->foot);
    S->active -= 1;
  }
}

// Completed batches: read results, free workspaces and slots.
bool harvest(hawkes_server* S) {
  bool any = false;
  for (auto& b : S->batches) {
    if (!b.busy) continue;
    bool complete;
    if (S->simulate) complete = now_ns() >= b.sim_done_ns;
    else complete = hipEventQuery(b.done) == hipSuccess;
    if (!complete) continue;
    for (int k = 0; k < b.nreq; ++k) {
      Request* r = b.reqs[k];
      if (S->simulate) {
        const double sim[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        finish(S, r, HAWKES_OK, sim);
      } else {
        const double* o = b.host_out + 8 * k;
        finish(S, r, (int)o[7], o);
      }
    }
    b.busy = false;
    b.reqs.clear();
    b.nreq = 0;
    any = true;
  }
  if (any) S->cv_done.notify_all();
  return any;
}

// Size band of a request: N within a factor of 4.  A batch completes when its
// largest request does, so mixing sizes would make small requests wait for a
// large one; banding keeps each batch's requests of similar duration, and the
// large ones run beside the small ones on other streams instead.
int size_band(int64_t n) {
  int b = 0;
  while (n >= 4) { n >>= 2; ++b; }
  return b;
}

// Admit from the FIFO into free batch slots and launch.  The head request
// decides the batch's class (D, precision, with or without a location
// gradient, size band); later requests of another class wait for a later
// batch.  D, precision and the gradient flag fix which kernels run, so a
// request's arithmetic is the same alone, in any batch and through the direct
// calls.  A head request that does not fit in memory blocks admission until
// memory frees up (no overtaking by smaller requests of its class), which
// keeps admission fair.
bool admit_and_launch(hawkes_server* S) {
  bool any = false;
  for (auto& b : S->batches) {
    if (b.busy || S->pending.empty()) continue;
    std::vector<Request*> take;
    int cls_d = -1, cls_p = -1, cls_b = -1;
    bool cls_g = false;
    for (auto it = S->pending.begin(); it != S->pending.end();) {
      Request* r = *it;
      const Dataset& ds = S->datasets[r->ds];
      if (S->active >= S->max_slots) break;
      if (cls_d < 0) { cls_d = ds.d; cls_p = r->prec; cls_g = r->grad_x != nullptr; cls_b = size_band(ds.n); }
      if (ds.d != cls_d || r->prec != cls_p || (r->grad_x != nullptr) != cls_g || size_band(ds.n) != cls_b) {
        ++it;
        continue;
      }
      size_t off;
      if (!S->arena.alloc(r->foot, &off)) {
        if (take.empty()) { cls_d = -1; }
        break;
      }
      r->off = off;
      r->admitted = true;
      r->res.t_admit_ns = now_ns();
      S->active += 1;
      take.push_back(r);
      it = S->pending.erase(it);
    }
    if (take.empty()) break;
    b.reqs = take;
    b.nreq = (int)take.size();
    b.busy = true;
    S->n_batches += 1;
    const uint64_t t0 = now_ns();
    for (auto* r : take) r->res.t_start_ns = t0;
    if (S->simulate) {
      // virtual device time: 1 ns per 1,000 ordered pairs plus 20 us
      double pairs = 0;
      for (auto* r : take) {
        const double n = (double)S->datasets[r->ds].n;
        pairs += n * (n - 1);
      }
      b.sim_done_ns = t0 + 20000 + (uint64_t)(pairs / 1000.0);
    } else {
      bool grad = false;
      for (int k = 0; k < b.nreq; ++k) {
        Request* r = take[k];
        const Dataset& ds = S->datasets[r->ds];
        Layout Lo;
        make_layout(ds.n, ds.d, r->prec, Lo);
        const KParams kp = make_kparams(Lo, &r->p);
        b.host_desc[k] = make_desc(Lo, kp, r->x, ds.t, S->arena_base + r->off, b.dev_out + 8 * k, r->grad_x);
        grad = grad || r->grad_x != nullptr;
      }
      const BatchGrid g = assign_blocks(b.host_desc, b.nreq);
      int st = HAWKES_OK;
      if (hipMemcpyAsync(b.dev_desc, b.host_desc, sizeof(ReqDesc) * b.nreq, hipMemcpyHostToDevice, b.stream) !=
          hipSuccess)
        st = HAWKES_EDEVICE;
      if (st == HAWKES_OK) st = launch_batch(cls_d, (cls_p & ~HAWKES_CULL) == HAWKES_MIXED, b.dev_desc, b.nreq, g, grad, b.stream);
      if (st == HAWKES_OK &&
          hipMemcpyAsync(b.host_out, b.dev_out, sizeof(double) * 8 * b.nreq, hipMemcpyDeviceToHost, b.stream) !=
              hipSuccess)
        st = HAWKES_EDEVICE;
      if (st == HAWKES_OK && hipEventRecord(b.done, b.stream) != hipSuccess) st = HAWKES_EDEVICE;
      if (st != HAWKES_OK) {
        // the launch failed: fail this batch's requests, keep serving others
        (void)hipStreamSynchronize(b.stream);
        for (auto* r : take) finish(S, r, st, nullptr);
        b.busy = false;
        b.reqs.clear();
        b.nreq = 0;
        S->cv_done.notify_all();
      }
    }
    any = true;
  }
  return any;
}

void worker_loop(hawkes_server* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    const bool h = harvest(S);
    const bool a = admit_and_launch(S);
    bool busy = false;
    for (auto& b : S->batches) busy = busy || b.busy;
    if (S->stop && S->pending.empty() && !busy) break;
    if (!h && !a) {
      // nothing changed: sleep until new work arrives, or briefly while
      // batches are in flight (their completion is polled)
      if (busy) S->cv_work.wait_for(lk, std::chrono::microseconds(20));
      else S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    }
  }
}

void free_server(hawkes_server* S) {
  for (auto& b : S->batches) {
    if (!S->simulate) {
      if (b.stream) (void)hipStreamDestroy(b.stream);
      if (b.done) (void)hipEventDestroy(b.done);
      dev_free(S, b.dev_desc);
      dev_free(S, b.dev_out);
      if (b.host_desc) (void)hipHostFree(b.host_desc);
      if (b.host_out) (void)hipHostFree(b.host_out);
    }
  }
  if (!S->simulate) {
    for (auto& ds : S->datasets)
      dev_free(S, ds.t);
    dev_free(S, S->arena_base);
  }
  for (auto& kv : S->by_ticket) delete kv.second;
  delete S;
}

}  // namespace
}  // namespace hawkes

extern "C" {

size_t hawkes_serve_footprint(int64_t n, int d, int prec) { return hawkes::footprint(n, d, prec); }

int hawkes_serve_create(size_t hbm_budget_bytes, int max_slots, int flags, hawkes_server_t** out) {
  return hawkes_serve_create_with(nullptr, hbm_budget_bytes, max_slots, flags, out);
}

int hawkes_serve_create_with(const hawkes_allocator_t* alloc, size_t hbm_budget_bytes, int max_slots, int flags,
                             hawkes_server_t** out) {
  using namespace hawkes;
  if (!out || max_slots < 1 || max_slots > 1024 || hbm_budget_bytes < (1u << 20)) return HAWKES_EINVAL;
  if (alloc && (!alloc->alloc || !alloc->free)) return HAWKES_EINVAL;
  const int streams = std::max(1, std::min(8, flags & 0xff ? (flags & 0xff) : 2));
  hawkes_server* S = new hawkes_server;
  if (alloc) S->alloc = *alloc;
  S->budget = hbm_budget_bytes;
  S->max_slots = max_slots;
  S->simulate = (flags & HAWKES_SERVE_SIMULATE) != 0;
  S->arena.reset(hbm_budget_bytes);
  S->batches.resize(streams);
  if (!S->simulate) {
    S->arena_base = static_cast<char*>(dev_alloc(S, hbm_budget_bytes));
    bool ok = S->arena_base != nullptr;
    for (auto& b : S->batches) {
      ok = ok && hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) == hipSuccess;
      ok = ok && hipEventCreateWithFlags(&b.done, hipEventDisableTiming) == hipSuccess;
      ok = ok && (b.dev_desc = static_cast<ReqDesc*>(dev_alloc(S, sizeof(ReqDesc) * max_slots))) != nullptr;
      ok = ok && (b.dev_out = static_cast<double*>(dev_alloc(S, sizeof(double) * 8 * max_slots))) != nullptr;
      ok = ok && hipHostMalloc(&b.host_desc, sizeof(ReqDesc) * max_slots, hipHostMallocDefault) == hipSuccess;
      ok = ok && hipHostMalloc(&b.host_out, sizeof(double) * 8 * max_slots, hipHostMallocDefault) == hipSuccess;
    }
    if (!ok) {
      free_server(S);
      return HAWKES_EDEVICE;
    }
  } else {
    for (auto& b : S->batches) {
      b.host_desc = nullptr;
      b.host_out = nullptr;
    }
  }
  S->worker = std::thread(worker_loop, S);
  *out = S;
  return HAWKES_OK;
}

int hawkes_serve_register(hawkes_server_t* S, const double* t, int64_t n, int d, int32_t* dataset_id) {
  using namespace hawkes;
  if (!S || !t || !dataset_id) return HAWKES_EINVAL;
  Layout Lo;
  if (!make_layout(n, d, HAWKES_MIXED, Lo)) return HAWKES_EINVAL;
  Dataset ds;
  ds.n = n;
  ds.d = d;
  if (!S->simulate) {
    ds.t = static_cast<double*>(dev_alloc(S, sizeof(double) * n));
    if (!ds.t) return HAWKES_EDEVICE;
    if (hipMemcpy(ds.t, t, sizeof(double) * n, hipMemcpyDeviceToDevice) != hipSuccess) {
      dev_free(S, ds.t);
      return HAWKES_EDEVICE;
    }
  } else {
    ds.t = const_cast<double*>(t);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) {
    if (!S->simulate) dev_free(S, ds.t);
    return HAWKES_ESTATE;
  }
  S->datasets.push_back(ds);
  *dataset_id = (int32_t)S->datasets.size() - 1;
  return HAWKES_OK;
}

int hawkes_serve_submit(hawkes_server_t* S, int32_t dataset_id, const double* x, const hawkes_params_t* p, int prec,
                        double* grad_x, uint64_t* ticket) {
  using namespace hawkes;
  if (!S || !x || !p || !ticket) return HAWKES_EINVAL;
  if ((prec & ~HAWKES_CULL) != HAWKES_FP64 && (prec & ~HAWKES_CULL) != HAWKES_MIXED) return HAWKES_EINVAL;
  if (!valid_params(p)) return HAWKES_EPARAM;
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return HAWKES_ESTATE;
  if (dataset_id < 0 || dataset_id >= (int32_t)S->datasets.size()) return HAWKES_ESTATE;
  const Dataset& ds = S->datasets[dataset_id];
  const size_t foot = footprint(ds.n, ds.d, prec);
  if (foot == 0) return HAWKES_EINVAL;
  if (foot > S->arena.capacity()) return HAWKES_ENOMEM;
  auto* r = new Request;
  r->ticket = S->next_ticket++;
  r->ds = dataset_id;
  r->x = x;
  r->p = *p;
  r->prec = prec;
  r->grad_x = grad_x;
  r->foot = foot;
  r->res.status = HAWKES_EPENDING;
  r->res.t_submit_ns = now_ns();
  S->pending.push_back(r);
  S->by_ticket[r->ticket] = r;
  S->n_requests += 1;
  *ticket = r->ticket;
  S->cv_work.notify_one();
  return HAWKES_OK;
}

int hawkes_serve_poll(hawkes_server_t* S, uint64_t ticket, hawkes_result_t* out) {
  if (!S || !out) return HAWKES_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->by_ticket.find(ticket);
  if (it == S->by_ticket.end()) return HAWKES_ESTATE;
  if (!it->second->done) return HAWKES_EPENDING;
  *out = it->second->res;
  delete it->second;
  S->by_ticket.erase(it);
  return HAWKES_OK;
}

int hawkes_serve_wait(hawkes_server_t* S, uint64_t ticket, hawkes_result_t* out, int64_t timeout_ns) {
  if (!S || !out) return HAWKES_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->by_ticket.find(ticket);
  if (it == S->by_ticket.end()) return HAWKES_ESTATE;
  hawkes::Request* r = it->second;
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns < 0 ? 0 : timeout_ns);
  while (!r->done) {
    if (timeout_ns >= 0 && S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !r->done)
      return HAWKES_ETIMEOUT;
    if (timeout_ns < 0) S->cv_done.wait(lk);
  }
  *out = r->res;
  delete r;
  S->by_ticket.erase(ticket);
  return HAWKES_OK;
}

int hawkes_serve_stats(hawkes_server_t* S, hawkes_serve_stats_t* out) {
  if (!S || !out) return HAWKES_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  out->pending = (int64_t)S->pending.size();
  out->active = S->active;
  out->batches_launched = S->n_batches;
  out->requests_submitted = S->n_requests;
  out->arena_bytes = S->arena.capacity();
  out->arena_free_bytes = S->arena.free_bytes();
  return HAWKES_OK;
}

int hawkes_serve_destroy(hawkes_server_t* S) {
  if (!S) return HAWKES_EINVAL;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  hawkes::free_server(S);
  return HAWKES_OK;
}

}  // extern "C"
