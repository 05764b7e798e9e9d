// Host-side internals shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mlmq.h"
#include "mlmq_internal.h"

// Device-resident graph (the opaque mlmq_graph of the C ABI).
struct mlmq_graph {
  int32_t n = 0;
  int64_t m = 0;
  int32_t* d_off = nullptr;   // [n+1]
  uint64_t* d_adj = nullptr;  // [m] col | weight << 32
  // degree-ordered copy (power-law graphs, for plain solves): vertex v is
  // vertex ord_of[v] there; null when the graph keeps its order
  int32_t* d_off_ord = nullptr;
  uint64_t* d_adj_ord = nullptr;
  uint32_t* d_ord_of = nullptr;     // [n] on the device
  std::vector<uint32_t> h_ord_of;   // [n] on the host (sources)
  mlmq_features features{};
  uint64_t deg_hist[33]{};    // bucket k: degrees in [2^(k-1), 2^k), bucket 0: degree 0
  uint32_t max_w = 0;
  uint32_t min_w = 0;
  bool overflow_safe = false;  // (n-1) * max_w < 2^32 - 1
  std::mutex mu;
  bool has_tuned = false;
  mlmq_config tuned{};
  int32_t sel_template = -1;  // the selector's top template (-1: the feature heuristic)
};

namespace mlmq {

struct DeviceInfo {
  bool ok = false;
  int device = 0;
  int cus = 0;
  uint64_t ticks_per_ms = 100000;
  size_t lds_per_wg = 65536;
  char name[64] = {0};
};

// Byte layout of one query's queue memory inside a slab.
struct QueryPlan {
  uint32_t nrings = 1, nb_log2 = 4, hub_cap = 1, init_words = 0;
  size_t off_ctrl = 0, off_rings = 0, off_hdr = 0, off_data = 0, off_hub_rec = 0, off_hub_cur = 0, off_hub_pub = 0;
  size_t bytes = 0;
};

// A reusable device allocation plus a pinned host staging area.
struct Slab {
  void* dev = nullptr;
  size_t dev_bytes = 0;
  void* host = nullptr;
  size_t host_bytes = 0;
  hipGraphExec_t graph_exec = nullptr;  // cached captured launch (batch)
  std::vector<uint64_t> graph_key;      // every argument baked into graph_exec
};

struct LaunchShape {
  uint32_t wg = 256, waves = 4, l1_cap = 64, grid = 1, max_grid = 1;
  bool two = false;
  bool stage = false;
  bool pq = false;  // kernel variant with the L2 priority-queue code
  size_t lds = 0;
};

extern thread_local std::string g_last_error;
int set_error(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
const DeviceInfo* device_info();
int need_device();
int check_config(const mlmq_config* c);
void default_config(mlmq_config* c);
void heuristic_config(const mlmq_graph* g, mlmq_config* c);
// Candidate template t (-1: the feature heuristic) as a config for g.
int template_config(const mlmq_graph* g, int32_t t, mlmq_config* out);
// The selector's top template for a graph with features f (-1 without a trained model).
int32_t selector_pick(const mlmq_features& f);
const mlmq_config* resolve_config(const mlmq_graph* g, const mlmq_config* cfg, mlmq_config* tmp);
uint64_t count_degree_above(const mlmq_graph* g, uint32_t th);
QueryPlan plan_query(const mlmq_graph* g, const mlmq_config& c, uint32_t extra_nb_log2, uint32_t hub_scale);
QueryDesc make_desc(const mlmq_graph* g, const mlmq_config& c, const QueryPlan& p, char* base, uint32_t* dist,
                    uint32_t source, uint32_t want_wgs);
int slab_acquire(size_t dev_bytes, size_t host_bytes, Slab** out);
void slab_release(Slab* s);
void pool_trim();
int launch_shape(const mlmq_config& c, uint32_t l1_cap, bool two, bool stage, bool pq, LaunchShape* out);
LaunchArgs make_args(const QueryDesc* d_desc, BatchCtrl* d_batch, int nq, const LaunchShape& s, uint32_t timeout_ms,
                     uint32_t* d_beats);
int status_to_code(uint32_t st);
std::string describe_query_state(const QueryDesc& d, const uint32_t* d_beats, uint32_t nbeats);
void fill_stats(mlmq_stats* st, const QueryCtrl& h, double ms, double worker_ms, uint32_t grid, uint32_t retries);
int run_single(const mlmq_graph* g, uint32_t source, uint32_t* dist_out, const mlmq_config& c,
               bool unit_weights = false);
// What the host watchdog snapshots when a launch overruns its deadline.
struct WatchdogView {
  const QueryCtrl* d_ctrl = nullptr;  // first query's control block
  const RingCtr* d_rings = nullptr;   // its ring counters
  const uint32_t* d_beats = nullptr;  // per-wave heartbeats
  uint32_t nbeats = 0;
};
// side: the stream that carries the snapshot reads and the cancel store
// (nullptr = a library stream created on first use).
hipError_t wait_with_watchdog(hipStream_t stream, uint32_t timeout_ms, uint32_t* d_cancel, uint32_t* h_one,
                              const WatchdogView& view, hipStream_t side = nullptr);

}  // namespace mlmq
