// Serving: continuous batching of independent decompositions.
//
// rlu_serve_start allocates one HBM pool and `max_inflight` slots (a HIP
// stream of default priority, an auxiliary stream and a completion event
// each).  rlu_submit validates and plans a request and queues it.  A worker
// thread admits queued requests whenever a slot is free and the pool has room
// for the request's workspace and the device for its LU panel blocks
// (serve_policy.h: first fit, oldest first,
// younger ones may pass a head that does not fit a bounded number of times),
// enqueues the request's whole stage sequence on the slot's stream, and
// retires it when the slot's event completes, returning its workspace to the
// pool.  Requests of different shapes therefore run concurrently on the
// device, and a request that arrives while others are running starts as soon
// as memory and a slot free up.  Sketches and intermediate factors live in
// the pool, outputs in the caller's device buffers.  rlu_poll retires
// finished tickets.
//
// LU panels, whose blocks wait for each other, are ordinary launches
// instead of cooperative ones (which leave the device idle for about 11 us
// around each panel): a request is admitted only while the panel blocks of
// all running requests, its own included, number at most one per compute
// unit, which keeps every waiting block's siblings placeable.
//
// One slot (max_inflight = 1): requests run one at a time, and each
// request's stage sequence is captured into a HIP graph on the slot stream
// and launched as one graph.  The slot keeps the instantiated graphs of
// recent launch topologies and updates one in place (hipGraphExecUpdate) for
// a request with the same topology.  The stages run in order on the slot
// stream, so a graph is one chain of nodes.  With more slots, requests share
// the device and their stages are enqueued directly.
#include <algorithm>
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
constexpr int kGraphCache = 16;  // instantiated graphs kept per slot

// Launch topology of a captured request: its nodes in capture order, each as
// (node type, kernel function).  Requests of different shapes often launch
// the same kernel sequence with other grids and arguments, which an
// instantiated graph takes by hipGraphExecUpdate, so the topology, not the
// shape, is the cache key.
struct GraphEntry {
  uint64_t hash = 0;
  std::vector<uint64_t> topo;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};

static bool graph_topology(hipGraph_t g, std::vector<uint64_t> *topo, uint64_t *hash) {
  size_t n = 0;
  if (hipGraphGetNodes(g, nullptr, &n) != hipSuccess) return false;
  std::vector<hipGraphNode_t> nodes(n);
  if (n && hipGraphGetNodes(g, nodes.data(), &n) != hipSuccess) return false;
  topo->assign(2 * n, 0);
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the words
  for (size_t i = 0; i < n; ++i) {
    hipGraphNodeType t;
    if (hipGraphNodeGetType(nodes[i], &t) != hipSuccess) return false;
    uint64_t f = 0;
    if (t == hipGraphNodeTypeKernel) {
      hipKernelNodeParams kp{};
      if (hipGraphKernelNodeGetParams(nodes[i], &kp) != hipSuccess) return false;
      f = (uint64_t)reinterpret_cast<uintptr_t>(kp.func);
    }
    (*topo)[2 * i] = (uint64_t)t;
    (*topo)[2 * i + 1] = f;
    for (uint64_t w : {(uint64_t)t, f}) {
      h ^= w;
      h *= 1099511628211ull;
    }
  }
  *hash = h;
  return true;
}

struct ServeRequest {
  uint64_t ticket;
  rlu_matrix A;
  rlu_params p;
  rlu_factors out;
  FactorPlan fp;
  size_t bytes;
  int blocks = 0;  // blocks of the request's widest LU panel launch
  int bypassed = 0;
};

struct ServeSlot {
  hipStream_t st = nullptr;
  AuxStream ax;            // auxiliary stream (same compute units) and its fork / join events
  hipEvent_t done = nullptr;
  std::vector<GraphEntry> graphs;
  bool busy = false;
  uint64_t ticket = 0;
  size_t off = 0, bytes = 0;
  int blocks = 0;
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
  bool exclusive_slot = false;  // one slot with the device to itself: exclusive panels, graphs
  DevCaps caps{};          // what the requests are planned for
  uint64_t launches = 0;
  uint64_t graph_hits = 0, graph_builds = 0, graph_fallbacks = 0;
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

// One request's stage sequence on its slot.  On the single exclusive slot:
// captured into a graph and launched as one (an instantiated graph of the
// slot updated in place when the topology allows, else a new one, the least
// recently used dropped); if capture fails the stages are enqueued directly.
static rlu_status launch_request(ServeState *s, ServeSlot &sl, const ServeRequest &r, void *ws) {
  ExecEnv env;
  env.caps = s->caps;
  env.ax = sl.ax;
  // LU panels are ordinary launches, not cooperative ones: the blocks of a
  // panel wait for each other, and admission keeps the panel blocks of all
  // running requests within one per compute unit, so while any panel block
  // waits for a sibling not yet placed, some compute unit holds no waiting
  // block and frees up as its other work ends.  (The waits are also bounded
  // in time and end in RLU_ERR_TIMEOUT.)
  env.exclusive = true;
  env.overlap = !s->exclusive_slot;
  if (!s->exclusive_slot) return factor_enqueue(*s->cx, &r.A, &r.p, &r.out, ws, r.fp, sl.st, &env);
  ++s->launches;
  hipError_t e = hipStreamBeginCapture(sl.st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ++s->graph_fallbacks;
    return factor_enqueue(*s->cx, &r.A, &r.p, &r.out, ws, r.fp, sl.st, &env);
  }
  const rlu_status st = factor_enqueue(*s->cx, &r.A, &r.p, &r.out, ws, r.fp, sl.st, &env);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(sl.st, &g);
  if (st != RLU_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (st != RLU_OK) return st;
    ++s->graph_fallbacks;
    return factor_enqueue(*s->cx, &r.A, &r.p, &r.out, ws, r.fp, sl.st, &env);
  }
  std::vector<uint64_t> topo;
  uint64_t hash = 0;
  if (!graph_topology(g, &topo, &hash)) {
    (void)hipGetLastError();
    topo.clear();
    hash = 0;  // an entry that no later topology matches
  }
  GraphEntry *hit = nullptr;
  for (GraphEntry &ge : sl.graphs)
    if (!topo.empty() && ge.hash == hash && ge.topo == topo) { hit = &ge; break; }
  hipGraphExec_t exec = nullptr;
  if (hit) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateError;
    if (hipGraphExecUpdate(hit->exec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
      exec = hit->exec;
      ++s->graph_hits;
    } else {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(hit->exec);
      hit->exec = nullptr;
    }
  }
  if (!exec) {
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      (void)hipGraphDestroy(g);
      if (hit) sl.graphs.erase(sl.graphs.begin() + (hit - sl.graphs.data()));
      ++s->graph_fallbacks;
      return factor_enqueue(*s->cx, &r.A, &r.p, &r.out, ws, r.fp, sl.st, &env);
    }
    ++s->graph_builds;
    if (!hit) {
      if ((int)sl.graphs.size() >= kGraphCache) {
        size_t lru = 0;
        for (size_t i = 1; i < sl.graphs.size(); ++i)
          if (sl.graphs[i].last_use < sl.graphs[lru].last_use) lru = i;
        (void)hipGraphExecDestroy(sl.graphs[lru].exec);
        sl.graphs.erase(sl.graphs.begin() + lru);
      }
      sl.graphs.push_back(GraphEntry{hash, std::move(topo), nullptr, 0});
      hit = &sl.graphs.back();
    }
    hit->exec = exec;
  }
  hit->last_use = s->launches;
  (void)hipGraphDestroy(g);
  e = hipGraphLaunch(exec, sl.st);
  return e == hipSuccess ? RLU_OK : hip_fail(e, "hipGraphLaunch");
}

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
      // LU panel blocks of the running requests: together at most one per
      // compute unit (see launch_request)
      int held = 0;
      for (const ServeSlot &o : s->slots) held += o.busy ? o.blocks : 0;
      const int idx = serve::pick_next(s->queue, s->alloc, s->caps.num_cu - held, kMaxBypass, &off);
      if (idx < 0) break;
      ServeRequest r = s->queue[idx];
      s->queue.erase(s->queue.begin() + idx);
      sl.busy = true;
      sl.ticket = r.ticket;
      sl.off = off;
      sl.bytes = r.bytes;
      sl.blocks = r.blocks;
      ++s->running;
      s->tickets[r.ticket].state = kRunning;
      lk.unlock();  // launching does not hold up rlu_submit / rlu_poll
      rlu_status st = launch_request(s, sl, r, s->pool + off);
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
    if (sl.st) (void)hipStreamSynchronize(sl.st);
    if (sl.ax.aux && sl.ax.aux != sl.st) (void)hipStreamSynchronize(sl.ax.aux);
    for (GraphEntry &ge : sl.graphs)
      if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
    sl.graphs.clear();
    if (sl.ax.aux && sl.ax.aux != sl.st) (void)hipStreamDestroy(sl.ax.aux);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.ax.fork) (void)hipEventDestroy(sl.ax.fork);
    if (sl.ax.join) (void)hipEventDestroy(sl.ax.join);
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
  s->caps = cx.caps;
  s->exclusive_slot = max_inflight == 1;  // the one slot has the device to itself
  for (ServeSlot &sl : s->slots) {
    e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
    if (e == hipSuccess) {
      if (s->exclusive_slot) sl.ax.aux = sl.st;  // its stages run in order on the slot stream
      else e = hipStreamCreateWithFlags(&sl.ax.aux, hipStreamNonBlocking);
    }
    sl.ax.main = sl.st;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ax.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ax.join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e != hipSuccess) {
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
  if ((st = plan_factor(s->caps, A, p, &r.fp)) != RLU_OK) return st;
  r.A = *A;
  r.p = *p;
  r.out = *out;
  r.bytes = r.fp.total;
  r.blocks = std::max(r.fp.py.G, r.fp.pb.G);
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

rlu_status rlu_serve_stats(rlu_ctx *ctx, uint64_t *stats) {
  if (!ctx || !stats) return fail(RLU_ERR_INVALID_ARG, "NULL argument");
  ServeState *s = reinterpret_cast<rlu_ctx_impl *>(ctx)->serve;
  if (!s) return fail(RLU_ERR_INVALID_ARG, "serving not started (rlu_serve_start)");
  std::lock_guard<std::mutex> g(s->mu);
  stats[0] = s->exclusive_slot ? 1u : 0u;
  stats[1] = (uint64_t)s->caps.num_cu;
  stats[2] = s->launches;
  stats[3] = s->graph_hits;
  stats[4] = s->graph_builds;
  stats[5] = s->graph_fallbacks;
  stats[6] = stats[7] = 0;
  return RLU_OK;
}

rlu_status rlu_serve_stop(rlu_ctx *ctx) {
  if (!ctx) return fail(RLU_ERR_INVALID_ARG, "ctx is NULL");
  return stop_state(*reinterpret_cast<rlu_ctx_impl *>(ctx));
}

}  // extern "C"
