// Continuous-batching server: a resident persistent kernel serves queries
// from a slot table while the host admits new ones as slots and memory free
// up. The queue system of each query is the same as a plain solve's, so each
// result is identical to the query's solve alone.
//
// Host thread loop:
//   1. completions: the last wave to leave a query writes (status, generation)
//      into host-coherent memory; the host retires the query (capacity errors
//      are retried with a doubled L2, graphs that may overflow 32 bits get the
//      exact overflow check), and frees its slot and memory;
//   2. admission, in arrival order: a free slot and a pool range for the
//      query's queues must exist and the per-query state (queues + distances)
//      must fit in the memory budget; the init kernel and the slot-opening
//      kernel go to a control stream that runs beside the resident kernel;
//   3. liveness: resident waves leave after a stretch without work, so when
//      queries are in flight and the kernel has fully exited, it is launched
//      again.
// Device-wide synchronisation (hipDeviceSynchronize) waits for the resident
// kernel, so a caller must not use it while a server is alive; both streams
// are non-blocking, so work on the null stream does not wait for them.

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "mlmq_api_internal.h"

using namespace mlmq;

namespace {

constexpr uint64_t kSlotClosedBit = 1ull << 31;
constexpr size_t kMaxPending = 1u << 20;
// Fewest waves a query gets while the server is busy (a single solve is
// latency-bound well before it fills the device).
constexpr uint32_t kMinShare = 128;

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over one device range (host bookkeeping only).
class RangePool {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      return true;
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

 private:
  std::map<size_t, size_t> free_;
};

struct Request {
  int32_t graph = 0;
  uint32_t source = 0;
  uint32_t* dist = nullptr;
  uint64_t submit_ns = 0, done_ns = 0;
  int32_t status = 1;  // 1 = not finished
  uint32_t extra = 0, hub_scale = 1, retries = 0;
};

enum class Phase { kFree, kRun, kCheck };

struct Slot {
  Phase phase = Phase::kFree;
  uint64_t ticket = 0;
  uint32_t gen = 0;
  size_t off = 0, bytes = 0, charge = 0;
  hipEvent_t ev = nullptr;
};

}  // namespace

struct mlmq_server {
  std::vector<const mlmq_graph*> graphs;
  std::vector<mlmq_config> cfgs;
  std::vector<uint32_t> want;
  int32_t nslots = 0;
  uint64_t budget = 0, charged = 0;

  char* d_pool = nullptr;
  RangePool pool;
  QueryDesc* d_slots = nullptr;
  uint64_t* d_join = nullptr;
  ServerCtrl* d_ctl = nullptr;
  uint64_t* h_done = nullptr;  // host-coherent
  uint32_t* h_ovf = nullptr;   // host-coherent, one word per slot
  hipStream_t ws = nullptr, cs = nullptr;
  ServerArgs args{};
  uint32_t grid = 0;
  size_t lds = 0;

  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool quit = false;
  std::string fatal;
  std::deque<uint64_t> pending;
  std::vector<Request> reqs;  // ticket t is reqs[t - 1]
  std::vector<Slot> slots;
  uint32_t next_gen = 1;
  uint32_t launches = 0;
  uint32_t timeout_ms = 60000;
  uint64_t quit_ns = 0;
  bool cancel_sent = false;
  bool leak = false;  // the device never let go of the server's memory
  bool stopping = false;        // stop flag raised on an idle server, kernel not yet gone
  uint64_t last_active_ns = 0;  // last time a query was pending or running
};

namespace {

size_t query_charge(const mlmq_server* s, const Request& r, QueryPlan* plan) {
  *plan = plan_query(s->graphs[r.graph], s->cfgs[r.graph], r.extra, r.hub_scale);
  return plan->bytes + 4ull * s->graphs[r.graph]->n;
}

void finish(mlmq_server* s, uint64_t t, int32_t status) {
  Request& r = s->reqs[t - 1];
  r.status = status;
  r.done_ns = now_ns();
  s->cv_done.notify_all();
}

void free_slot(mlmq_server* s, Slot& sl) {
  s->pool.release(sl.off, sl.bytes);
  s->charged -= sl.charge;
  sl.phase = Phase::kFree;
  sl.ticket = 0;
}

// Fails every query still pending or in flight (device error or shutdown).
void fail_all(mlmq_server* s, int32_t code) {
  for (uint64_t t : s->pending) finish(s, t, code);
  s->pending.clear();
  for (Slot& sl : s->slots)
    if (sl.phase != Phase::kFree) {
      finish(s, sl.ticket, code);
      free_slot(s, sl);
    }
}

// Retires finished queries; returns true if anything changed.
bool collect(mlmq_server* s) {
  bool any = false;
  for (int32_t i = 0; i < s->nslots; ++i) {
    Slot& sl = s->slots[i];
    if (sl.phase == Phase::kRun) {
      const uint64_t w = __atomic_load_n(&s->h_done[i], __ATOMIC_ACQUIRE);
      if ((uint32_t)w != sl.gen) continue;
      any = true;
      const uint32_t st = (uint32_t)(w >> 32) & 0xFFu, ovf = (uint32_t)(w >> 40) & 1u;
      Request& r = s->reqs[sl.ticket - 1];
      const mlmq_graph* g = s->graphs[r.graph];
      if ((st == kStCapacity || st == kStHubCapacity) && r.retries < s->cfgs[r.graph].max_retries) {
        if (st == kStCapacity) r.extra += 1;
        else r.hub_scale *= 4;
        r.retries += 1;
        s->pending.push_front(sl.ticket);
        free_slot(s, sl);
        continue;
      }
      const int code = status_to_code(st);
      if (code == MLMQ_OK && ovf && !g->overflow_safe) {
        // exact check (a candidate overflowed; the result may still fit)
        s->h_ovf[i] = 0;
        hipError_t e = launch_overflow_check(s->d_slots + i, s->h_ovf + i, s->cs);
        if (e == hipSuccess) e = hipEventRecord(sl.ev, s->cs);
        if (e != hipSuccess) {
          finish(s, sl.ticket, MLMQ_ERR_DEVICE);
          free_slot(s, sl);
          continue;
        }
        sl.phase = Phase::kCheck;
        continue;
      }
      finish(s, sl.ticket, code);
      free_slot(s, sl);
    } else if (sl.phase == Phase::kCheck) {
      const hipError_t e = hipEventQuery(sl.ev);
      if (e == hipErrorNotReady) continue;
      any = true;
      const uint32_t flag = __atomic_load_n(&s->h_ovf[i], __ATOMIC_ACQUIRE);
      finish(s, sl.ticket, e != hipSuccess ? MLMQ_ERR_DEVICE : (flag ? MLMQ_ERR_DISTANCE_OVERFLOW : MLMQ_OK));
      free_slot(s, sl);
    }
  }
  return any;
}

// Admits pending queries in arrival order; returns true if any was admitted.
bool admit(mlmq_server* s, std::string* err) {
  bool any = false;
  while (!s->pending.empty()) {
    int32_t free_i = -1;
    for (int32_t i = 0; i < s->nslots; ++i)
      if (s->slots[i].phase == Phase::kFree) {
        free_i = i;
        break;
      }
    if (free_i < 0) break;
    const uint64_t t = s->pending.front();
    Request& r = s->reqs[t - 1];
    QueryPlan plan;
    const size_t charge = query_charge(s, r, &plan);
    if (s->charged + charge > s->budget && s->charged > 0) break;
    size_t off = 0;
    const size_t bytes = (plan.bytes + 255) & ~size_t(255);
    if (!s->pool.alloc(bytes, &off)) {
      if (s->charged == 0) {  // can never fit
        s->pending.pop_front();
        finish(s, t, MLMQ_ERR_OUT_OF_MEMORY);
        continue;
      }
      break;
    }
    s->pending.pop_front();
    Slot& sl = s->slots[free_i];
    const mlmq_graph* g = s->graphs[r.graph];
    // Wave share: the graph's own launch size when the server is quiet, an
    // equal split of the resident waves (at least kMinShare) when it is busy.
    uint32_t busy = 1 + (uint32_t)std::min<size_t>(s->pending.size(), 64);
    for (const Slot& o : s->slots) busy += o.phase == Phase::kRun ? 1u : 0u;
    const uint32_t want = std::max(std::min(s->want[r.graph], s->grid / busy), std::min(kMinShare, s->want[r.graph]));
    const QueryDesc d = make_desc(g, s->cfgs[r.graph], plan, s->d_pool + off, r.dist, r.source, want);
    const uint32_t gen = s->next_gen++;
    if (s->next_gen == 0) s->next_gen = 1;
    __atomic_store_n(&s->h_done[free_i], 0ull, __ATOMIC_RELEASE);
    const uint64_t word = ((uint64_t)gen << 32) | ((uint64_t)want << 16);
    const hipError_t e =
        launch_server_admit(d, s->d_slots + free_i, s->d_join + free_i, word, plan.init_words, s->cs);
    if (e != hipSuccess) {
      s->pool.release(off, bytes);
      finish(s, t, MLMQ_ERR_DEVICE);
      *err = std::string("admission launch: ") + hipGetErrorString(e);
      return any;
    }
    sl.phase = Phase::kRun;
    sl.ticket = t;
    sl.gen = gen;
    sl.off = off;
    sl.bytes = bytes;
    sl.charge = charge;
    s->charged += charge;
    any = true;
  }
  return any;
}

bool in_flight(const mlmq_server* s) {
  for (const Slot& sl : s->slots)
    if (sl.phase == Phase::kRun) return true;
  return false;
}

// Launches the resident kernel if queries are running and no wave is left.
hipError_t keep_alive(mlmq_server* s) {
  if (!in_flight(s)) return hipSuccess;
  const hipError_t q = hipStreamQuery(s->ws);
  if (q == hipErrorNotReady) return hipSuccess;
  if (q != hipSuccess) return q;
  s->launches += 1;
  return launch_server_worker(s->args, s->grid, s->lds, s->ws);
}

// The resident kernel leaves as a whole: after kIdleStopNs without pending
// or running queries the host raises the stop flag and admits nothing until
// the kernel is gone; the flag is cleared on the worker stream, ahead of the
// next launch. (Waves leaving one by one would leave a thin kernel that the
// host does not relaunch, and later queries would run on a few waves.)
constexpr uint64_t kIdleStopNs = 200ull * 1000000ull;

hipError_t idle_stop(mlmq_server* s) {
  const uint64_t now = now_ns();
  const bool quiet = !in_flight(s) && s->pending.empty();
  if (!quiet || !s->last_active_ns) s->last_active_ns = now;
  if (!s->stopping && quiet && now - s->last_active_ns > kIdleStopNs && hipStreamQuery(s->ws) == hipErrorNotReady) {
    const hipError_t e = launch_server_signal(&s->d_ctl->stop.v, 1u, s->cs);
    if (e != hipSuccess) return e;
    s->stopping = true;
  }
  if (s->stopping && hipStreamQuery(s->ws) == hipSuccess) {
    const hipError_t e = launch_server_signal(&s->d_ctl->stop.v, 0u, s->ws);
    if (e != hipSuccess) return e;
    s->stopping = false;
  }
  return hipSuccess;
}

void server_loop(mlmq_server* s) {
  (void)hipSetDevice(device_info()->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    std::string err;
    bool any = collect(s);
    if (!s->quit) {
      const hipError_t ie = idle_stop(s);
      if (ie != hipSuccess) err = std::string("idle stop: ") + hipGetErrorString(ie);
      if (err.empty() && !s->stopping) any |= admit(s, &err);
    }
    hipError_t e = err.empty() ? keep_alive(s) : hipErrorUnknown;
    if (e != hipSuccess) {
      s->fatal = err.empty() ? std::string("resident kernel: ") + hipGetErrorString(e) : err;
      fail_all(s, MLMQ_ERR_DEVICE);
      return;
    }
    if (s->quit) {
      for (uint64_t t : s->pending) finish(s, t, MLMQ_ERR_CANCELED);
      s->pending.clear();
      bool busy = false;
      for (const Slot& sl : s->slots) busy |= sl.phase != Phase::kFree;
      if (!busy) return;
      // running queries end at their device deadline; past it (plus slack),
      // cancel them, and if even that is not answered, give up on the memory
      const uint64_t now = now_ns();
      if (!s->quit_ns) s->quit_ns = now;
      const uint64_t grace = (uint64_t)(s->timeout_ms + 5000) * 1000000ull;
      if (!s->cancel_sent && now - s->quit_ns > grace) {
        s->cancel_sent = true;
        (void)launch_server_signal(&s->d_ctl->cancel.v, 1u, s->cs);
      }
      if (now - s->quit_ns > grace + 5000000000ull) {
        s->leak = true;
        fail_all(s, MLMQ_ERR_TIMEOUT);
        return;
      }
    }
    if (!any) s->cv_work.wait_for(lk, std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

int mlmq_server_create(const mlmq_graph* const* graphs, int32_t ngraphs, uint64_t mem_budget_bytes,
                       int32_t max_slots, const mlmq_config* cfg, mlmq_server** out) {
  if (!out || !graphs || ngraphs < 1) return set_error(MLMQ_ERR_INVALID_ARG, "graphs and out are required");
  if (max_slots < 1 || max_slots > 64) return set_error(MLMQ_ERR_INVALID_ARG, "max_slots must be in [1, 64]");
  if (mem_budget_bytes == 0) return set_error(MLMQ_ERR_INVALID_ARG, "mem_budget_bytes must be positive");
  for (int32_t i = 0; i < ngraphs; ++i)
    if (!graphs[i]) return set_error(MLMQ_ERR_INVALID_ARG, "graph %d is NULL", i);
  int rc = need_device();
  if (rc) return rc;
  if (cfg && (rc = check_config(cfg))) return rc;

  auto* s = new mlmq_server();
  s->nslots = max_slots;
  s->budget = mem_budget_bytes;
  uint32_t l1_alloc = 64;
  bool two = false, stage = false, pq = false;
  uint32_t timeout_ms = 0;
  for (int32_t i = 0; i < ngraphs; ++i) {
    mlmq_config tmp;
    const mlmq_config* c = resolve_config(graphs[i], cfg, &tmp);
    mlmq_config cc = *c;
    cc.stream = nullptr;
    cc.stats_out = nullptr;
    s->graphs.push_back(graphs[i]);
    s->cfgs.push_back(cc);
    if (cc.l1_type != MLMQ_L1_NONE) l1_alloc = std::max(l1_alloc, cc.l1_cap);
    two |= cc.l1_type == MLMQ_L1_NEARFAR;
    stage |= cc.l2_type == MLMQ_L2_BUCKET;
    pq |= cc.l2_type == MLMQ_L2_PQ;
    timeout_ms = std::max(timeout_ms, cc.timeout_ms);
  }
  auto fail = [&](int code) {
    mlmq_server_destroy(s);
    return code;
  };
  const DeviceInfo* di = device_info();
  s->lds = worker_lds_bytes(1, l1_alloc, two, stage);
  if (s->lds > di->lds_per_wg) return fail(set_error(MLMQ_ERR_INVALID_ARG, "L1 does not fit in LDS"));
  int per_cu = 0;
  hipError_t e = server_occupancy(s->lds, pq, &per_cu);
  if (e != hipSuccess) return fail(hip_fail(e, "occupancy query"));
  if (per_cu < 1) return fail(set_error(MLMQ_ERR_INVALID_ARG, "server kernel does not fit on a CU"));
  // One workgroup per CU fewer than fit: the admission kernels (query init,
  // slot opening, overflow check) run beside the resident kernel, and when
  // registers rather than LDS bound its residency (power-law graphs with a
  // small L1: 3 waves per SIMD use 504 of 512 VGPRs) a full-size resident
  // grid would leave them no room until resident waves leave.
  s->grid = (uint32_t)std::max(1, per_cu - 1) * (uint32_t)di->cus;
  if (cfg && cfg->grid_wgs) s->grid = std::min(s->grid, cfg->grid_wgs);
  for (int32_t i = 0; i < ngraphs; ++i) {
    // at most the graph's own launch size (its config's grid_wgs, else all)
    uint32_t w = s->cfgs[i].grid_wgs ? std::min(s->grid, s->cfgs[i].grid_wgs) : s->grid;
    s->want.push_back(std::min<uint32_t>(std::max<uint32_t>(w, 1), 0x7FFF));
  }

  size_t max_plan = 0;
  for (int32_t i = 0; i < ngraphs; ++i)
    max_plan = std::max(max_plan, plan_query(graphs[i], s->cfgs[i], 0, 1).bytes);
  const size_t pool_bytes = std::max<size_t>(mem_budget_bytes, (max_plan + 255) & ~size_t(255));
  e = hipMalloc(reinterpret_cast<void**>(&s->d_pool), pool_bytes);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->d_slots), sizeof(QueryDesc) * 64);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->d_join), 8 * 64);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->d_ctl), sizeof(ServerCtrl));
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&s->h_done), 8 * 64, hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&s->h_ovf), 4 * 64, hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(set_error(MLMQ_ERR_OUT_OF_MEMORY, "server memory (%zu bytes)", pool_bytes));
  if (e != hipSuccess) return fail(hip_fail(e, "server memory"));
  s->pool.reset(pool_bytes);
  std::memset(s->h_done, 0, 8 * 64);
  std::memset(s->h_ovf, 0, 4 * 64);
  {
    std::vector<uint64_t> closed(64, kSlotClosedBit);
    ServerCtrl zero;
    std::memset(&zero, 0, sizeof(zero));
    e = hipMemcpy(s->d_join, closed.data(), 8 * 64, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->d_ctl, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(s->d_slots, 0, sizeof(QueryDesc) * 64);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->ws, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->cs, hipStreamNonBlocking);
  s->slots.resize(max_slots);
  for (Slot& sl : s->slots)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
  if (e != hipSuccess) return fail(hip_fail(e, "server setup"));

  ServerArgs& a = s->args;
  a.slots = s->d_slots;
  a.join = s->d_join;
  a.done_host = s->h_done;
  a.ctl = s->d_ctl;
  a.nslots = max_slots;
  a.l1_cap = l1_alloc;
  a.l1_two = two ? 1u : 0u;
  a.stage = stage ? 1u : 0u;
  a.pq = pq ? 1u : 0u;
  s->timeout_ms = timeout_ms ? timeout_ms : 60000;
  a.timeout_ticks = (uint64_t)s->timeout_ms * di->ticks_per_ms;
  a.cap_wait_ticks = 20ull * di->ticks_per_ms;
  a.idle_exit_ticks = 2000ull * di->ticks_per_ms;  // failsafe; the host stops an idle server after 200 ms
  s->th = std::thread(server_loop, s);
  *out = s;
  return MLMQ_OK;
}

int mlmq_server_submit(mlmq_server* s, int32_t graph_id, uint32_t source, uint32_t* dist_out, uint64_t* ticket) {
  if (!s || !ticket || !dist_out) return set_error(MLMQ_ERR_INVALID_ARG, "server, dist_out and ticket are required");
  if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size())
    return set_error(MLMQ_ERR_INVALID_ARG, "graph_id %d out of range", graph_id);
  if (source >= (uint32_t)s->graphs[graph_id]->n)
    return set_error(MLMQ_ERR_INVALID_ARG, "source %u out of range", source);
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->fatal.empty()) return set_error(MLMQ_ERR_DEVICE, "server failed: %s", s->fatal.c_str());
  if (s->quit) return set_error(MLMQ_ERR_CANCELED, "server is shutting down");
  if (s->pending.size() >= kMaxPending) return set_error(MLMQ_ERR_BUSY, "pending list full");
  Request r;
  r.graph = graph_id;
  r.source = source;
  r.dist = dist_out;
  r.submit_ns = now_ns();
  s->reqs.push_back(r);
  const uint64_t t = s->reqs.size();
  s->pending.push_back(t);
  *ticket = t;
  s->cv_work.notify_one();
  return MLMQ_OK;
}

int mlmq_server_poll(mlmq_server* s, uint64_t ticket, int32_t* done_status) {
  if (!s || !done_status) return set_error(MLMQ_ERR_INVALID_ARG, "server and done_status are required");
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket > s->reqs.size()) return set_error(MLMQ_ERR_INVALID_ARG, "unknown ticket");
  *done_status = s->reqs[ticket - 1].status;
  return MLMQ_OK;
}

int mlmq_server_wait(mlmq_server* s, uint64_t ticket, uint32_t timeout_ms) {
  if (!s) return set_error(MLMQ_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket > s->reqs.size()) return set_error(MLMQ_ERR_INVALID_ARG, "unknown ticket");
  const bool ok = s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                                      [&] { return s->reqs[ticket - 1].status != 1; });
  if (!ok) return set_error(MLMQ_ERR_TIMEOUT, "query %llu not finished", (unsigned long long)ticket);
  const int32_t st = s->reqs[ticket - 1].status;
  if (st != MLMQ_OK) return set_error(st, "query %llu failed (%d)", (unsigned long long)ticket, st);
  return MLMQ_OK;
}

int mlmq_server_times(mlmq_server* s, uint64_t ticket, uint64_t* submit_ns, uint64_t* done_ns) {
  if (!s || !submit_ns || !done_ns) return set_error(MLMQ_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket > s->reqs.size()) return set_error(MLMQ_ERR_INVALID_ARG, "unknown ticket");
  *submit_ns = s->reqs[ticket - 1].submit_ns;
  *done_ns = s->reqs[ticket - 1].done_ns;
  return MLMQ_OK;
}

void mlmq_server_destroy(mlmq_server* s) {
  if (!s) return;
  if (s->th.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->quit = true;
      s->cv_work.notify_one();
    }
    s->th.join();  // in-flight queries end (each is bounded by its device watchdog)
  }
  if (s->ws) {
    // idle waves leave on the stop flag; a wave still in a query leaves at its
    // deadline or on cancel
    if (s->d_ctl && s->cs && launch_server_signal(&s->d_ctl->stop.v, 1u, s->cs) == hipSuccess) {
      using clk = std::chrono::steady_clock;
      const auto limit = clk::now() + std::chrono::milliseconds(5000);
      while (hipStreamQuery(s->ws) == hipErrorNotReady && clk::now() < limit)
        std::this_thread::sleep_for(std::chrono::microseconds(200));
      if (hipStreamQuery(s->ws) == hipErrorNotReady) {
        (void)launch_server_signal(&s->d_ctl->cancel.v, 1u, s->cs);
        const auto limit2 = clk::now() + std::chrono::milliseconds(5000);
        while (hipStreamQuery(s->ws) == hipErrorNotReady && clk::now() < limit2)
          std::this_thread::sleep_for(std::chrono::microseconds(200));
      }
    }
  }
  if (s->cs) (void)hipStreamSynchronize(s->cs);
  if (s->leak || (s->ws && hipStreamQuery(s->ws) != hipSuccess)) {
    // a kernel may still touch this memory: keep it for the process lifetime
    delete s;
    return;
  }
  for (Slot& sl : s->slots)
    if (sl.ev) (void)hipEventDestroy(sl.ev);
  if (s->ws) (void)hipStreamDestroy(s->ws);
  if (s->cs) (void)hipStreamDestroy(s->cs);
  if (s->d_pool) (void)hipFree(s->d_pool);
  if (s->d_slots) (void)hipFree(s->d_slots);
  if (s->d_join) (void)hipFree(s->d_join);
  if (s->d_ctl) (void)hipFree(s->d_ctl);
  if (s->h_done) (void)hipHostFree(s->h_done);
  if (s->h_ovf) (void)hipHostFree(s->h_ovf);
  delete s;
}

}  // extern "C"
