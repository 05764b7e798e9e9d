// Batched solves in one persistent, hipGraph-captured launch.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mlmq.h"
#include "mlmq_api_internal.h"
#include "mlmq_internal.h"

using namespace mlmq;

namespace {

// Fewest waves a batched query is given when the batch is wide.
constexpr uint32_t kBatchShare = 128;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

hipStream_t internal_stream() {
  static hipStream_t s = nullptr;
  static std::once_flag once;
  std::call_once(once, [] { (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking); });
  return s;
}

bool device_ptr(const void* p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

}  // namespace

extern "C" int mlmq_sssp_batch(const mlmq_graph* const* graphs, const uint32_t* sources, uint32_t* const* dist_outs,
                               int32_t nq, const mlmq_config* const* cfgs, int32_t* per_query_status) {
  if (nq < 1 || !graphs || !sources || !dist_outs) return set_error(MLMQ_ERR_INVALID_ARG, "empty or NULL batch");
  int rc = need_device();
  if (rc) return rc;
  std::vector<mlmq_config> conf((size_t)nq);
  for (int32_t i = 0; i < nq; ++i) {
    if (!graphs[i]) return set_error(MLMQ_ERR_INVALID_ARG, "graphs[%d] is NULL", i);
    if (sources[i] >= (uint32_t)graphs[i]->n)
      return set_error(MLMQ_ERR_INVALID_ARG, "sources[%d] = %u out of range", i, sources[i]);
    if (!dist_outs[i] || !device_ptr(dist_outs[i]))
      return set_error(MLMQ_ERR_INVALID_ARG, "dist_outs[%d] must be device memory", i);
    mlmq_config tmp;
    conf[i] = *resolve_config(graphs[i], cfgs ? cfgs[i] : nullptr, &tmp);
    rc = check_config(&conf[i]);
    if (rc) return rc;
  }
  // Launch shape from the first config, but always the whole device: the
  // queries share it. LDS is sized for the largest L1.
  mlmq_config lc = conf[0];
  lc.grid_wgs = 0;
  uint32_t l1cap = 64;
  bool two = false, stage = false, pq = false;
  for (auto& c : conf) {
    if (c.l1_type != MLMQ_L1_NONE) l1cap = std::max(l1cap, c.l1_cap);
    two = two || c.l1_type == MLMQ_L1_NEARFAR;
    stage = stage || c.l2_type == MLMQ_L2_BUCKET;
    pq = pq || c.l2_type == MLMQ_L2_PQ;
  }
  LaunchShape shape;
  rc = launch_shape(lc, l1cap, two, stage, pq, &shape);
  if (rc) return rc;
  hipStream_t stream = lc.stream ? reinterpret_cast<hipStream_t>(lc.stream) : internal_stream();
  // Largest queries first, so the long ones start early (LPT order).
  std::vector<int32_t> order((size_t)nq);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return graphs[a]->m > graphs[b]->m; });
  // Queries in flight at once: each gets an equal share of the resident
  // waves (at least kBatchShare), capped by its own tuned launch size. A
  // single solve is latency-bound long before it fills the device, so many
  // narrow queries finish more work per second than a few wide ones.
  const uint32_t conc = (uint32_t)std::max<int64_t>(1, std::min<int64_t>(nq, shape.grid / kBatchShare));
  std::vector<QueryPlan> plans((size_t)nq);
  size_t bytes = 0;
  uint32_t init_words = 1;
  for (int32_t k = 0; k < nq; ++k) {
    const int32_t i = order[k];
    plans[k] = plan_query(graphs[i], conf[i], 0, 1);
    bytes = align_up(bytes + plans[k].bytes, 256);
    init_words = std::max(init_words, plans[k].init_words);
  }
  const size_t desc_off = bytes;
  const size_t batch_off = align_up(desc_off + sizeof(QueryDesc) * nq, 256);
  const size_t res_off = align_up(batch_off + sizeof(BatchCtrl), 256);
  const size_t beats_off = align_up(res_off + sizeof(QueryResult) * nq, 256);
  const size_t dev_bytes = align_up(beats_off + 4ull * shape.grid, 256);
  const size_t host_bytes = sizeof(QueryDesc) * nq + sizeof(QueryResult) * nq + 64;
  Slab* slab = nullptr;
  rc = slab_acquire(dev_bytes, host_bytes, &slab);
  if (rc) return rc;
  char* base = static_cast<char*>(slab->dev);
  QueryDesc* d_desc = reinterpret_cast<QueryDesc*>(base + desc_off);
  BatchCtrl* d_batch = reinterpret_cast<BatchCtrl*>(base + batch_off);
  QueryResult* d_res = reinterpret_cast<QueryResult*>(base + res_off);
  QueryDesc* h_desc = reinterpret_cast<QueryDesc*>(slab->host);
  QueryResult* h_res = reinterpret_cast<QueryResult*>(h_desc + nq);
  size_t off = 0;
  for (int32_t k = 0; k < nq; ++k) {
    const int32_t i = order[k];
    const mlmq_config& c = conf[i];
    const uint32_t share = std::max<uint32_t>(4, shape.grid / conc);
    const uint32_t want = c.grid_wgs ? std::min(c.grid_wgs, share) : share;
    h_desc[k] = make_desc(graphs[i], c, plans[k], base + off, dist_outs[i], sources[i], want);
    off = align_up(off + plans[k].bytes, 256);
  }
  uint32_t* d_beats = reinterpret_cast<uint32_t*>(base + beats_off);
  const LaunchArgs a = make_args(d_desc, d_batch, nq, shape, lc.timeout_ms, d_beats);
  // The captured launch bakes in every kernel argument: the launch shape and
  // the addresses of the descriptors, control words, results and heartbeats
  // (which move with the summed plan sizes of the queries before them). The
  // descriptors' contents are read at run time, so only these must match, and
  // they are compared in full (no hash).
  const std::vector<uint64_t> key = {(uint64_t)nq, (uint64_t)shape.grid, (uint64_t)shape.wg, (uint64_t)shape.lds,
                                     (uint64_t)init_words, (uint64_t)(uintptr_t)stream, a.timeout_ticks,
                                     a.cap_wait_ticks, (uint64_t)a.l1_cap, (uint64_t)a.l1_two, (uint64_t)a.stage,
                                     (uint64_t)a.waves, (uint64_t)(uintptr_t)d_desc, (uint64_t)(uintptr_t)d_batch,
                                     (uint64_t)(uintptr_t)d_res, (uint64_t)(uintptr_t)d_beats};
  hipError_t e = hipMemcpyAsync(d_desc, h_desc, sizeof(QueryDesc) * nq, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && (!slab->graph_exec || slab->graph_key != key)) {
    if (slab->graph_exec) {
      (void)hipGraphExecDestroy(slab->graph_exec);
      slab->graph_exec = nullptr;
    }
    // Capture init + persistent worker + result gather as one graph.
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e1 = launch_init(d_desc, d_batch, nq, init_words, stream);
      if (e1 == hipSuccess) e1 = launch_worker(a, shape.grid, shape.wg, shape.lds, stream);
      if (e1 == hipSuccess) e1 = launch_gather(d_desc, nq, d_res, stream);
      e = hipStreamEndCapture(stream, &graph);
      if (e == hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&slab->graph_exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e == hipSuccess) slab->graph_key = key;
  }
  if (e == hipSuccess) e = hipGraphLaunch(slab->graph_exec, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h_res, d_res, sizeof(QueryResult) * nq, hipMemcpyDeviceToHost, stream);
  uint32_t* h_one = reinterpret_cast<uint32_t*>(h_res + nq);
  WatchdogView view;
  view.d_ctrl = h_desc[0].ctrl;
  view.d_rings = h_desc[0].rings;
  view.d_beats = d_beats;
  view.nbeats = shape.grid;
  if (e == hipSuccess) e = wait_with_watchdog(stream, lc.timeout_ms, &d_batch->cancel.v, h_one, view);
  if (e == hipErrorLaunchTimeOut) {
    const std::string snap = g_last_error;
    if (hipStreamQuery(stream) == hipSuccess) slab_release(slab);
    return set_error(MLMQ_ERR_TIMEOUT, "device overran its timeout (%s)", snap.c_str());
  }
  if (e != hipSuccess) {
    slab_release(slab);
    return hip_fail(e, "batch launch");
  }
  int first_bad = MLMQ_OK;
  std::vector<int32_t> status((size_t)nq, MLMQ_OK);
  std::vector<int32_t> redo;
  for (int32_t k = 0; k < nq; ++k) {
    const int32_t i = order[k];
    int st = status_to_code(h_res[k].error);
    if (st == MLMQ_ERR_QUEUE_CAPACITY) {
      redo.push_back(i);  // solved again alone, with its own capacity retries
      continue;
    }
    if (st == MLMQ_OK && h_res[k].overflow && !graphs[i]->overflow_safe) redo.push_back(i);
    status[i] = st;
    if (cfgs && cfgs[i] && cfgs[i]->stats_out) {
      QueryCtrl tmp;
      std::memset(&tmp, 0, sizeof(tmp));
      tmp.error.v = h_res[k].error;
      for (int j = 0; j < kNumCounters; ++j) tmp.stats[j] = h_res[k].stats[j];
      fill_stats(cfgs[i]->stats_out, tmp, 0.0, 0.0, h_desc[k].want_wgs, 0);
    }
  }
  slab_release(slab);
  for (int32_t i : redo) {
    mlmq_config c = conf[i];
    c.stream = reinterpret_cast<void*>(stream);
    status[i] = run_single(graphs[i], sources[i], dist_outs[i], c);
  }
  for (int32_t i = 0; i < nq; ++i) {
    if (per_query_status) per_query_status[i] = status[i];
    if (status[i] != MLMQ_OK && first_bad == MLMQ_OK) first_bad = status[i];
  }
  if (first_bad != MLMQ_OK) set_error(first_bad, "at least one query of the batch failed");
  return first_bad;
}
