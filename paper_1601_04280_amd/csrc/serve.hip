// Serving: continuous batching of independent decompositions.
//
// rlu_serve_start allocates one HBM pool and `max_inflight` slots (a HIP
// stream of default priority and a completion event each).  rlu_submit
// validates and plans a request and queues it.  A worker thread admits
// queued requests whenever a slot is free and the pool has room for the
// request's workspace (serve_policy.h: first fit, oldest first, younger ones
// may pass a head that does not fit a bounded number of times), enqueues the
// request's whole stage sequence on the slot's stream, and retires it when the
// slot's event completes, returning its workspace to the pool.  Requests of
// different shapes therefore run concurrently on the device, and a request
// that arrives while others are running starts as soon as memory and a slot
// free up.  Sketches and intermediate factors live in the pool, outputs in
// the caller's device buffers.  rlu_poll retires finished tickets.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rlu_device.h"
#include "rlu_internal.h"
#include "serve_policy.h"

namespace rlu {

constexpr int kMaxInflight = 64;
constexpr int kMaxBypass = 8;

struct ServeRequest {
  uint64_t ticket;
  rlu_matrix A;
  rlu_params p;
  rlu_factors out;
  FactorPlan fp;
  size_t bytes;
  int bypassed = 0;
};

struct ServeSlot {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  uint64_t ticket = 0;
  size_t off = 0, bytes = 0;
  rlu_status status = RLU_OK;
  std::string msg;
};

enum TicketState { kQueued, kRunning, kDone };
struct TicketRec {
  TicketState state = kQueued;
  rlu_status status = RLU_OK;
  std::string msg;
};

struct ServeState {
  rlu_ctx_impl *cx = nullptr;
  char *pool = nullptr;
  serve::PoolAlloc alloc;
  std::vector<ServeSlot> slots;
  std::deque<ServeRequest> queue;
  std::unordered_map<uint64_t, TicketRec> tickets;
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stopping = false;
  int running = 0;
};

static void worker_main(ServeState *s) {
  (void)hipSetDevice(s->cx->caps.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progress = false;
    for (ServeSlot &sl : s->slots) {  // retire finished requests
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      TicketRec &t = s->tickets[sl.ticket];
      t.state = kDone;
      t.status = sl.status != RLU_OK ? sl.status : (q == hipSuccess ? RLU_OK : RLU_ERR_DEVICE);
      t.msg = sl.status != RLU_OK ? sl.msg : (q == hipSuccess ? "" : hipGetErrorString(q));
      s->alloc.release(sl.off, sl.bytes);
      sl.busy = false;
      --s->running;
      progress = true;
    }
    for (ServeSlot &sl : s->slots) {  // admit into free slots
      if (sl.busy) continue;
      size_t off = 0;
      const int idx = serve::pick_next(s->queue, s->alloc, kMaxBypass, &off);
      if (idx < 0) break;
      ServeRequest r = s->queue[idx];
      s->queue.erase(s->queue.begin() + idx);
      sl.busy = true;
      sl.ticket = r.ticket;
      sl.off = off;
      sl.bytes = r.bytes;
      ++s->running;
      s->tickets[r.ticket].state = kRunning;
      lk.unlock();  // launching does not hold up rlu_submit / rlu_poll
      rlu_status st = factor_enqueue(*s->cx, &r.A, &r.p, &r.out, s->pool + off, r.fp, sl.st);
      std::string msg = st != RLU_OK ? rlu_last_error() : "";
      const hipError_t e = hipEventRecord(sl.done, sl.st);
      if (st == RLU_OK && e != hipSuccess) {
        st = RLU_ERR_DEVICE;
        msg = std::string("hipEventRecord: ") + hipGetErrorString(e);
      }
      lk.lock();
      sl.status = st;
      sl.msg = msg;
      progress = true;
    }
    if (s->queue.empty() && s->running == 0) {
      if (s->stopping) break;
      s->cv.wait(lk);
      continue;
    }
    if (s->running == 0 && !progress) {
      // an empty pool that cannot take the oldest request: it never will
      for (const ServeRequest &r : s->queue) {
        TicketRec &t = s->tickets[r.ticket];
        t.state = kDone;
        t.status = RLU_ERR_NO_MEMORY;
        t.msg = "request does not fit the serving pool";
      }
      s->queue.clear();
      continue;
    }
    if (!progress) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(10));
      lk.lock();
    }
  }
}

static rlu_status stop_state(rlu_ctx_impl &cx) {
  ServeState *s = cx.serve;
  if (!s) return RLU_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stopping = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (ServeSlot &sl : s->slots) {
    if (sl.st) {
      (void)hipStreamSynchronize(sl.st);
      (void)hipStreamDestroy(sl.st);
    }
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  if (s->pool) (void)hipFree(s->pool);
  delete s;
  cx.serve = nullptr;
  return RLU_OK;
}

void serve_shutdown(rlu_ctx_impl &cx) { stop_state(cx); }

}  // namespace rlu

using namespace rlu;

extern "C" {

rlu_status rlu_serve_start(rlu_ctx *ctx, size_t hbm_budget_bytes, int max_inflight) {
  if (!ctx) return fail(RLU_ERR_INVALID_ARG, "ctx is NULL");
  rlu_ctx_impl &cx = *reinterpret_cast<rlu_ctx_impl *>(ctx);
  if (cx.serve) return fail(RLU_ERR_INVALID_ARG, "serving already started on this context");
  if (max_inflight < 1 || max_inflight > kMaxInflight)
    return fail(RLU_ERR_INVALID_ARG, "max_inflight must be in [1, %d]", kMaxInflight);
  if (hbm_budget_bytes < serve::kGranule) return fail(RLU_ERR_INVALID_ARG, "hbm_budget_bytes too small");
  hipError_t e = hipSetDevice(cx.caps.device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  ServeState *s = new (std::nothrow) ServeState();
  if (!s) return fail(RLU_ERR_NO_MEMORY, "host allocation failed");
  s->cx = &cx;
  const size_t bytes = hbm_budget_bytes / serve::kGranule * serve::kGranule;
  if ((e = hipMalloc(reinterpret_cast<void **>(&s->pool), bytes)) != hipSuccess) {
    (void)hipGetLastError();
    delete s;
    return fail(RLU_ERR_NO_MEMORY, "pool of %zu bytes: %s", bytes, hipGetErrorString(e));
  }
  s->alloc.reset(bytes);
  s->slots.resize(max_inflight);
  for (ServeSlot &sl : s->slots) {
    if ((e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess) {
      cx.serve = s;
      stop_state(cx);
      return hip_fail(e, "serving slot");
    }
  }
  cx.serve = s;
  try {
    s->worker = std::thread(worker_main, s);
  } catch (...) {
    stop_state(cx);
    return fail(RLU_ERR_NO_MEMORY, "could not start the serving thread");
  }
  return RLU_OK;
}

rlu_status rlu_submit(rlu_ctx *ctx, const rlu_matrix *A, const rlu_params *p, const rlu_factors *out,
                      uint64_t *ticket) {
  if (!ctx || !ticket) return fail(RLU_ERR_INVALID_ARG, "NULL argument");
  rlu_ctx_impl &cx = *reinterpret_cast<rlu_ctx_impl *>(ctx);
  ServeState *s = cx.serve;
  if (!s) return fail(RLU_ERR_INVALID_ARG, "serving not started (rlu_serve_start)");
  rlu_status st = validate_matrix(A);
  if (st != RLU_OK) return st;
  if ((st = validate_params(A, p)) != RLU_OK) return st;
  if ((st = validate_factors(A, p, out)) != RLU_OK) return st;
  if (p->flags & (RLU_FLAG_TIMING | RLU_FLAG_TIMING_CONTRACT))
    return fail(RLU_ERR_INVALID_ARG, "stage timing is not available for served requests");
  if (p->flags & RLU_FLAG_EXCLUSIVE)  // requests in flight share the device by design
    return fail(RLU_ERR_INVALID_ARG, "RLU_FLAG_EXCLUSIVE is not available for served requests");
  ServeRequest r;
  if ((st = plan_factor(cx, A, p, &r.fp)) != RLU_OK) return st;
  r.A = *A;
  r.p = *p;
  r.out = *out;
  r.bytes = r.fp.total;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stopping) return fail(RLU_ERR_INVALID_ARG, "serving is stopping");
    if (serve::round_up(r.bytes) > s->alloc.size())
      return fail(RLU_ERR_NO_MEMORY, "request needs %zu bytes of workspace; the pool holds %zu", r.bytes,
                  s->alloc.size());
    r.ticket = s->next_ticket++;
    s->tickets[r.ticket] = TicketRec{};
    s->queue.push_back(r);
    *ticket = r.ticket;
  }
  s->cv.notify_all();
  return RLU_OK;
}

rlu_status rlu_poll(rlu_ctx *ctx, uint64_t ticket) {
  if (!ctx) return fail(RLU_ERR_INVALID_ARG, "ctx is NULL");
  ServeState *s = reinterpret_cast<rlu_ctx_impl *>(ctx)->serve;
  if (!s) return fail(RLU_ERR_UNKNOWN_TICKET, "serving not started");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(RLU_ERR_UNKNOWN_TICKET, "no ticket %llu", (unsigned long long)ticket);
  if (it->second.state != kDone) return RLU_ERR_AGAIN;
  const rlu_status st = it->second.status;
  const std::string msg = it->second.msg;
  s->tickets.erase(it);
  return st == RLU_OK ? RLU_OK : fail(st, "%s", msg.c_str());
}

rlu_status rlu_serve_stop(rlu_ctx *ctx) {
  if (!ctx) return fail(RLU_ERR_INVALID_ARG, "ctx is NULL");
  return stop_state(*reinterpret_cast<rlu_ctx_impl *>(ctx));
}

}  // extern "C"
