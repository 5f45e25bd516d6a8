// cs_serve.cpp -- the queued request server (cs_queue_*): continuous batching
// of action computations on one GPU.
//
// A server thread owns S slots, each with its own HIP stream.  Requests are
// admitted in arrival order whenever a slot is free and their device
// footprint (matrix N*W*8 + coordinates + sort scratch + count workspace)
// fits under the context budget; resident matrices of idle requests are
// evicted least-recently-used to make room.  An admitted request runs
// sprinkle -> sort -> link -> count -> reduce on its slot's stream, so
// requests in different slots overlap on the device.  Finished matrices stay
// resident (up to the resident budget), keyed by (d, N, seed): a repeated
// request skips sprinkling and linking.  The result (integer counts, one
// rounding for the action) does not depend on what else runs.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "cs_internal.h"
#include "cs_runtime.h"

namespace cs {

using Clock = std::chrono::steady_clock;

struct Resident {
  std::tuple<int, int64_t, uint64_t> key;
  uint64_t* bits = nullptr;
  size_t bytes = 0;
  int users = 0;  // active requests reading it
  // Set when the request that sprinkled and linked it has finished without
  // error.  Until then another request must not read it: its link may still
  // be running on the producer's stream, and a 4D matrix whose acceptance
  // fell short is discarded and built again.
  bool ready = false;
};

struct Request {
  uint64_t ticket = 0;
  cs_req req{};
  Clock::time_point t_submit, t_admit, t_done;
  bool done = false;
  int redo = 0;  // 4D: times the acceptance fell short (each doubles the candidates)
  cs_result res{};
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
  std::shared_ptr<Request> rq;
  Resident* res = nullptr;        // matrix used by the running request
  std::vector<void*> transient;   // coords, scratch, workspace
  uint64_t* host = nullptr;       // pinned: 6 stats words + accepted count
  int64_t ncand = 0;
};

struct QueueState {
  cs_ctx* ctx = nullptr;
  uint64_t resident_budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> pending;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
  std::deque<uint64_t> completed;  // finished, not yet returned, in completion order
  std::list<std::unique_ptr<Resident>> resident;  // most recent first
  uint64_t resident_bytes = 0;
  std::vector<Slot> slots;
  uint64_t next_ticket = 1;
  int64_t outstanding = 0;
  std::atomic<bool> stop{false};
  std::thread th;
};

static void delete_queue_state(QueueState* q) { delete q; }

static size_t footprint(int d, int64_t N, int64_t ncand, bool need_matrix) {
  const size_t W = (size_t)row_words(N);
  size_t b = (size_t)N * d * 8 + (size_t)N * 8 + sprinkle_scratch_bytes(d, N, ncand) +
             (size_t)std::max<int64_t>(num_row_blocks(N), 1) * 6 * 8 + 6 * 8;
  if (need_matrix) b += (size_t)N * W * 8 + link_workspace_bytes(d, N);
  return b + 5 * 256;
}

static Resident* find_resident(QueueState* q, const std::tuple<int, int64_t, uint64_t>& key) {
  for (auto it = q->resident.begin(); it != q->resident.end(); ++it) {
    if ((*it)->key == key) {
      q->resident.splice(q->resident.begin(), q->resident, it);
      return q->resident.front().get();
    }
  }
  return nullptr;
}

// Evict idle resident matrices (LRU first) until `need` more bytes fit.
static bool make_room(QueueState* q, size_t need) {
  Pool& pool = q->ctx->pool;
  while (pool.live_bytes + need > pool.budget) {
    Resident* victim = nullptr;
    for (auto it = q->resident.rbegin(); it != q->resident.rend(); ++it)
      if ((*it)->users == 0) {
        victim = it->get();
        break;
      }
    if (!victim) return false;
    pool.release(victim->bits);
    q->resident_bytes -= victim->bytes;
    q->resident.remove_if([&](const std::unique_ptr<Resident>& r) { return r.get() == victim; });
  }
  return true;
}

static void finish_request(QueueState* q, Slot& s, cs_status st) {
  Request& r = *s.rq;
  r.t_done = Clock::now();
  r.res.status = st;
  if (st == CS_OK) {
    for (int k = 0; k < 4; ++k) r.res.n[k] = s.host[k];
    r.res.R = s.host[4];
    r.res.summ = s.host[5];
    r.res.S = bd_action(r.req.d, r.req.N, r.res.n);
  }
  r.done = true;
  q->completed.push_back(r.ticket);
  for (void* p : s.transient) q->ctx->pool.release(p);
  s.transient.clear();
  if (s.res) {
    s.res->users--;
    if (st == CS_OK) s.res->ready = true;
    if (st != CS_OK && s.res->users == 0) {
      // a failed request's matrix is never reused
      Resident* bad = s.res;
      q->ctx->pool.release(bad->bits);
      q->resident_bytes -= bad->bytes;
      q->resident.remove_if([&](const std::unique_ptr<Resident>& x) { return x.get() == bad; });
    }
    // keep it resident only while the resident budget allows
    while (q->resident_bytes > q->resident_budget) {
      Resident* victim = nullptr;
      for (auto it = q->resident.rbegin(); it != q->resident.rend(); ++it)
        if ((*it)->users == 0) {
          victim = it->get();
          break;
        }
      if (!victim) break;
      q->ctx->pool.release(victim->bits);
      q->resident_bytes -= victim->bytes;
      q->resident.remove_if([&](const std::unique_ptr<Resident>& x) { return x.get() == victim; });
    }
  }
  s.res = nullptr;
  s.busy = false;
  s.rq.reset();
  q->outstanding--;
}

// Launch one admitted request on slot s.  Returns false if memory did not fit.
static bool launch_request(QueueState* q, Slot& s, std::shared_ptr<Request> rq, int path) {
  cs_ctx* ctx = q->ctx;
  const int d = rq->req.d;
  const int64_t N = rq->req.N;
  const int64_t W = row_words(N);
  const auto key = std::make_tuple(d, N, rq->req.seed);
  Resident* res = find_resident(q, key);
  // the same matrix is still being built by an earlier request: wait for it
  // (the caller keeps this request at the head of the queue)
  if (res && !res->ready) return false;
  const int64_t ncand = d == 4 ? candidates_4d(N) << rq->redo : N;
  const size_t need = footprint(d, N, ncand, res == nullptr);
  if (!make_room(q, need)) return false;
  std::vector<void*> tr;
  auto grab = [&](size_t b) {
    void* p = ctx->pool.alloc(b);
    if (p) tr.push_back(p);
    return p;
  };
  uint64_t* ws = (uint64_t*)grab((size_t)std::max<int64_t>(num_row_blocks(N), 1) * 6 * 8);
  uint64_t* tot = (uint64_t*)grab(8 * 8);
  uint64_t* bits = res ? res->bits : nullptr;
  bool ok = ws && tot;
  double* coords = nullptr;
  int64_t* orig = nullptr;
  void* scratch = nullptr;
  void* ltab = nullptr;
  if (ok && !res) {
    coords = (double*)grab((size_t)N * d * 8);
    orig = (int64_t*)grab((size_t)N * 8);
    scratch = grab(sprinkle_scratch_bytes(d, N, ncand));
    const size_t lb = link_workspace_bytes(d, N);
    if (lb) ltab = grab(lb);
    bits = (uint64_t*)ctx->pool.alloc((size_t)N * W * 8);
    ok = coords && orig && scratch && bits && (ltab || !lb);
  }
  if (!ok) {
    for (void* p : tr) ctx->pool.release(p);
    if (!res && bits) ctx->pool.release(bits);
    return false;
  }
  if (!res) {
    auto r = std::make_unique<Resident>();
    r->key = key;
    r->bits = bits;
    r->bytes = (size_t)N * W * 8;
    q->resident.push_front(std::move(r));
    res = q->resident.front().get();
    q->resident_bytes += res->bytes;
  }
  res->users++;
  s.res = res;
  s.transient = tr;
  s.rq = rq;
  s.busy = true;
  s.ncand = ncand;
  rq->t_admit = Clock::now();
  hipStream_t st = s.stream;
  const bool fresh = coords != nullptr;
  hipError_t e = hipSuccess;
  s.host[6] = (uint64_t)N;  // accepted count, overwritten for 4D
  if (fresh && N > 0) {
    e = launch_sprinkle(d, N, rq->req.seed, ncand, coords, orig, scratch, tot + 6, st);
    if (e == hipSuccess) e = launch_link(d, N, coords, bits, W, ltab, st);
  }
  if (e == hipSuccess) e = launch_fill_u64(ws, 0, (size_t)std::max<int64_t>(num_row_blocks(N), 1) * 6, st);
  if (e == hipSuccess && N > 1) e = run_count(bits, N, W, 3, path, ws, st);
  if (e == hipSuccess) e = launch_reduce_rows(ws, std::max<int64_t>(num_row_blocks(N), 1), 3, tot, st);
  if (e == hipSuccess) e = hipMemcpyAsync(s.host, tot, 6 * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && fresh && d == 4 && N > 0)
    e = hipMemcpyAsync(s.host + 6, tot + 6, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(s.ev, st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    finish_request(q, s, CS_EDEVICE);
  }
  return true;
}

static void server(QueueState* q) {
  cs_ctx* ctx = q->ctx;
  (void)hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(q->mu);
  while (!q->stop.load()) {
    bool progressed = false;
    // completions
    for (Slot& s : q->slots) {
      if (!s.busy) continue;
      hipError_t e = hipEventQuery(s.ev);
      if (e == hipErrorNotReady) continue;
      progressed = true;
      if (e != hipSuccess) {
        (void)hipGetLastError();
        finish_request(q, s, CS_EDEVICE);
        continue;
      }
      Request& r = *s.rq;
      if (r.req.d == 4 && (int64_t)s.host[6] < r.req.N) {
        // far tail of the 4D acceptance: redo this request from scratch with
        // twice the candidates (the same counters, so the same first N)
        Resident* bad = s.res;
        std::shared_ptr<Request> again = s.rq;
        if (again->redo >= 7) {
          finish_request(q, s, CS_EDEVICE);
          continue;
        }
        again->redo++;
        for (void* p : s.transient) ctx->pool.release(p);
        s.transient.clear();
        bad->users--;
        ctx->pool.release(bad->bits);
        q->resident_bytes -= bad->bytes;
        q->resident.remove_if([&](const std::unique_ptr<Resident>& x) { return x.get() == bad; });
        s.res = nullptr;
        s.busy = false;
        s.rq.reset();
        q->pending.push_front(again);  // still outstanding
        continue;
      }
      finish_request(q, s, CS_OK);
    }
    if (progressed) q->cv_done.notify_all();
    // admissions, in arrival order
    while (!q->pending.empty()) {
      Slot* free_slot = nullptr;
      for (Slot& s : q->slots)
        if (!s.busy) {
          free_slot = &s;
          break;
        }
      if (!free_slot) break;
      std::shared_ptr<Request> rq = q->pending.front();
      const int d = rq->req.d;
      const int64_t N = rq->req.N;
      lk.unlock();
      const int path = N > 1 ? tuned_path(ctx, d, N) : CS_PATH_POP;  // may time kernels once
      lk.lock();
      const bool launched = launch_request(q, *free_slot, rq, path);
      if (!launched) {
        bool any_busy = false;
        for (Slot& s : q->slots) any_busy |= s.busy;
        if (!any_busy) {
          // cannot fit even on an idle device: fail it
          q->pending.pop_front();
          rq->t_admit = rq->t_done = Clock::now();
          rq->res = cs_result{};
          rq->res.status = CS_ENOMEM;
          rq->done = true;
          q->completed.push_back(rq->ticket);
          q->outstanding--;
          q->cv_done.notify_all();
          continue;
        }
        break;  // wait for a running request to free memory
      }
      q->pending.pop_front();
      progressed = true;
    }
    bool any_busy = false;
    for (Slot& s : q->slots) any_busy |= s.busy;
    if (!progressed) {
      if (any_busy) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      } else {
        q->cv_work.wait_for(lk, std::chrono::milliseconds(50));
      }
    }
  }
}

}  // namespace cs

using namespace cs;

extern "C" {

cs_status cs_queue_start(cs_ctx* ctx, int slots, uint64_t resident_budget) {
  if (!ctx || slots < 1 || slots > 64) return fail(CS_EINVAL, "cs_queue_start: slots must be 1..64");
  if (ctx->queue) return fail(CS_EBUSY, "cs_queue_start: already running");
  (void)hipSetDevice(ctx->device);
  auto* q = new QueueState();
  q->ctx = ctx;
  q->resident_budget = resident_budget ? resident_budget : ctx->pool.budget;
  q->slots.resize((size_t)slots);
  for (Slot& s : q->slots) {
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&s.host, 8 * 8) != hipSuccess) {
      for (Slot& t : q->slots) {
        if (t.stream) (void)hipStreamDestroy(t.stream);
        if (t.ev) (void)hipEventDestroy(t.ev);
        if (t.host) (void)hipHostFree(t.host);
      }
      delete q;
      return fail(CS_EDEVICE, "cs_queue_start: stream/event/pinned allocation failed");
    }
  }
  ctx->queue = std::unique_ptr<QueueState, void (*)(QueueState*)>(q, delete_queue_state);
  q->th = std::thread(server, q);
  return CS_OK;
}

cs_status cs_queue_submit(cs_ctx* ctx, const cs_req* req, uint64_t* ticket) {
  if (!ctx || !req || !ticket) return fail(CS_EINVAL, "cs_queue_submit: NULL argument");
  if (!ctx->queue) return fail(CS_EINVAL, "cs_queue_submit: queue not started");
  if ((req->d != 2 && req->d != 4) || req->N < 0 || req->N > ((int64_t)1 << 31))
    return fail(CS_EINVAL, "cs_queue_submit: bad request (d=%d, N=%lld)", req->d, (long long)req->N);
  QueueState* q = ctx->queue.get();
  auto r = std::make_shared<Request>();
  r->req = *req;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> g(q->mu);
    r->ticket = q->next_ticket++;
    q->all[r->ticket] = r;
    q->pending.push_back(r);
    q->outstanding++;
  }
  q->cv_work.notify_one();
  *ticket = r->ticket;
  return CS_OK;
}

cs_status cs_queue_poll(cs_ctx* ctx, uint64_t ticket, cs_result* out, double* timing) {
  if (!ctx || !out) return fail(CS_EINVAL, "cs_queue_poll: NULL argument");
  if (!ctx->queue) return fail(CS_EINVAL, "cs_queue_poll: queue not started");
  QueueState* q = ctx->queue.get();
  std::lock_guard<std::mutex> g(q->mu);
  auto it = q->all.find(ticket);
  if (it == q->all.end()) return fail(CS_EINVAL, "cs_queue_poll: unknown ticket %llu", (unsigned long long)ticket);
  Request& r = *it->second;
  if (!r.done) return CS_EBUSY;
  *out = r.res;
  if (timing) {
    using sec = std::chrono::duration<double>;
    timing[0] = sec(r.t_admit - r.t_submit).count();
    timing[1] = sec(r.t_done - r.t_admit).count();
    timing[2] = sec(r.t_done - r.t_submit).count();
  }
  q->all.erase(it);
  return CS_OK;
}

cs_status cs_queue_next(cs_ctx* ctx, double timeout_s, uint64_t* ticket, cs_result* out,
                        double* timing) {
  if (!ctx || !ticket || !out) return fail(CS_EINVAL, "cs_queue_next: NULL argument");
  if (!ctx->queue) return fail(CS_EINVAL, "cs_queue_next: queue not started");
  QueueState* q = ctx->queue.get();
  std::unique_lock<std::mutex> lk(q->mu);
  const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                        std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 0.0));
  for (;;) {
    // tickets already returned by cs_queue_poll are gone from `all`
    while (!q->completed.empty() && !q->all.count(q->completed.front())) q->completed.pop_front();
    if (!q->completed.empty()) break;
    if (timeout_s <= 0 || q->cv_done.wait_until(lk, until) == std::cv_status::timeout) {
      while (!q->completed.empty() && !q->all.count(q->completed.front())) q->completed.pop_front();
      if (q->completed.empty()) return CS_EBUSY;
      break;
    }
  }
  const uint64_t t = q->completed.front();
  q->completed.pop_front();
  auto it = q->all.find(t);
  Request& r = *it->second;
  *ticket = t;
  *out = r.res;
  if (timing) {
    using sec = std::chrono::duration<double>;
    timing[0] = sec(r.t_admit - r.t_submit).count();
    timing[1] = sec(r.t_done - r.t_admit).count();
    timing[2] = sec(r.t_done - r.t_submit).count();
  }
  q->all.erase(it);
  return CS_OK;
}

cs_status cs_queue_drain(cs_ctx* ctx) {
  if (!ctx) return fail(CS_EINVAL, "cs_queue_drain: NULL context");
  if (!ctx->queue) return CS_OK;
  QueueState* q = ctx->queue.get();
  std::unique_lock<std::mutex> lk(q->mu);
  q->cv_done.wait(lk, [&] { return q->outstanding == 0; });
  return CS_OK;
}

cs_status cs_queue_stop(cs_ctx* ctx) {
  if (!ctx || !ctx->queue) return CS_OK;
  QueueState* q = ctx->queue.get();
  q->stop.store(true);
  q->cv_work.notify_all();
  if (q->th.joinable()) q->th.join();
  for (Slot& s : q->slots) {
    (void)hipStreamSynchronize(s.stream);
    for (void* p : s.transient) ctx->pool.release(p);
    if (s.res) s.res->users--;
    (void)hipStreamDestroy(s.stream);
    (void)hipEventDestroy(s.ev);
    (void)hipHostFree(s.host);
  }
  for (auto& r : q->resident) ctx->pool.release(r->bits);
  q->resident.clear();
  ctx->queue.reset();
  return CS_OK;
}

}  // extern "C"
