// C ABI of the MLMQ SSSP library: graph residency, configuration, single and
// batched solves, graph features and the empirical autotuner.
//
// Every step of a solve runs in the HIP kernels of mlmq_kernels.hip; this file
// validates arguments, owns device memory and launches.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mlmq.h"
#include "mlmq_api_internal.h"
#include "mlmq_internal.h"

using namespace mlmq;

namespace mlmq {

thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return set_error(e == hipErrorOutOfMemory ? MLMQ_ERR_OUT_OF_MEMORY : MLMQ_ERR_DEVICE, "%s: %s", what,
                   hipGetErrorString(e));
}

// ------------------------------------------------------------ device info

const DeviceInfo* device_info() {
  static std::once_flag once;
  static DeviceInfo info;
  std::call_once(once, [] {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
      (void)hipGetLastError();
      info.ok = false;
      return;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
      info.ok = false;
      return;
    }
    info.ok = true;
    info.device = dev;
    info.cus = p.multiProcessorCount;
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate_khz <= 0)
      rate_khz = 100000;
    info.ticks_per_ms = (uint64_t)rate_khz;
    info.lds_per_wg = (size_t)p.sharedMemPerBlock;
    snprintf(info.name, sizeof(info.name), "%s", p.gcnArchName);
  });
  return &info;
}

int need_device() {
  const DeviceInfo* d = device_info();
  if (!d->ok) return set_error(MLMQ_ERR_DEVICE, "no HIP device available");
  return MLMQ_OK;
}

// ------------------------------------------------------------ configuration

static bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }
static uint32_t log2_ceil(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

int check_config(const mlmq_config* c) {
  if (!c) return set_error(MLMQ_ERR_INVALID_ARG, "config is NULL");
  if (c->struct_size != sizeof(mlmq_config))
    return set_error(MLMQ_ERR_INVALID_ARG, "config struct_size %u != %zu", c->struct_size, sizeof(mlmq_config));
  if (c->l0_rows > kMaxL0Rows) return set_error(MLMQ_ERR_INVALID_ARG, "l0_rows must be 0..%d", kMaxL0Rows);
  if (c->l1_type > MLMQ_L1_SLF) return set_error(MLMQ_ERR_INVALID_ARG, "unknown l1_type %u", c->l1_type);
  if (c->l2_type > MLMQ_L2_PQ) return set_error(MLMQ_ERR_INVALID_ARG, "unknown l2_type %u", c->l2_type);
  if (c->l2_type == MLMQ_L2_PQ && (c->pnum < 1 || c->pnum > 64))
    return set_error(MLMQ_ERR_INVALID_ARG, "pnum must be in [1, 64]");
  if (c->relax_mode > MLMQ_RELAX_ATOMIC)
    return set_error(MLMQ_ERR_INVALID_ARG, "unknown relax_mode %u", c->relax_mode);
  if (c->l1_type != MLMQ_L1_NONE && (!is_pow2(c->l1_cap) || c->l1_cap < 64 || c->l1_cap > 8192))
    return set_error(MLMQ_ERR_INVALID_ARG, "l1_cap must be a power of two in [64, 8192]");
  if (c->delta1 < 1) return set_error(MLMQ_ERR_INVALID_ARG, "delta1 must be >= 1");
  if (c->delta2_log2 > 31) return set_error(MLMQ_ERR_INVALID_ARG, "delta2_log2 must be <= 31");
  if (c->l2_type == MLMQ_L2_BUCKET && (!is_pow2(c->bmax) || c->bmax < 2 || c->bmax > (uint32_t)kMaxBuckets))
    return set_error(MLMQ_ERR_INVALID_ARG, "bmax must be a power of two in [2, %d]", kMaxBuckets);
  if (c->l2_type == MLMQ_L2_BUCKET && (c->bnum < 1 || c->bnum > c->bmax))
    return set_error(MLMQ_ERR_INVALID_ARG, "bnum must be in [1, bmax]");
  if (c->hub_chunk < 64 || c->hub_chunk % 64)
    return set_error(MLMQ_ERR_INVALID_ARG, "hub_chunk must be a positive multiple of 64");
  if (c->th_hub && c->th_hub < c->hub_chunk)
    return set_error(MLMQ_ERR_INVALID_ARG, "th_hub must be 0 or >= hub_chunk");
  if (c->wg_size != 64) return set_error(MLMQ_ERR_INVALID_ARG, "wg_size must be 64 (one wave per workgroup)");
  if (c->l2_capacity > (1ull << 34)) return set_error(MLMQ_ERR_INVALID_ARG, "l2_capacity too large");
  if (c->donate_min && (c->donate_min < 16 || c->donate_min > 65536))
    return set_error(MLMQ_ERR_INVALID_ARG, "donate_min must be 0 or in [16, 65536]");
  return MLMQ_OK;
}

void default_config(mlmq_config* c) {
  mlmq_stats* keep_stats = c->stats_out;
  void* keep_stream = c->stream;
  std::memset(c, 0, sizeof(*c));
  c->struct_size = sizeof(mlmq_config);
  c->l0_rows = 2;
  c->l1_type = MLMQ_L1_VEC;
  c->l2_type = MLMQ_L2_FIFO;
  c->l1_cap = 1024;
  c->l1_flush_wb = 64;
  c->delta1 = 256;
  c->delta2_log2 = 7;
  c->bmax = 32;
  c->bnum = 4;
  c->th_v = 32;
  c->th_hub = 8192;
  c->hub_chunk = 2048;
  c->wg_size = 64;
  c->grid_wgs = 0;
  c->l2_capacity = 0;
  c->timeout_ms = 60000;
  c->max_retries = 3;
  c->pnum = 1;
  c->stats_out = keep_stats;
  c->stream = keep_stream;
}

// ------------------------------------------------------------ graph

static int validate_csr(int32_t n, int64_t m, const int32_t* off, const int32_t* col) {
  if (n < 1) return set_error(MLMQ_ERR_INVALID_ARG, "n must be >= 1");
  if (m < 0 || m >= (1ll << 31)) return set_error(MLMQ_ERR_INVALID_ARG, "m must be in [0, 2^31)");
  if (!off || (m > 0 && !col)) return set_error(MLMQ_ERR_INVALID_ARG, "CSR pointer is NULL");
  if (off[0] != 0) return set_error(MLMQ_ERR_INVALID_ARG, "row_offsets[0] != 0");
  for (int32_t u = 0; u < n; ++u)
    if (off[u + 1] < off[u]) return set_error(MLMQ_ERR_INVALID_ARG, "row_offsets decrease at %d", u);
  if ((int64_t)off[n] != m) return set_error(MLMQ_ERR_INVALID_ARG, "row_offsets[n] != m");
  for (int64_t e = 0; e < m; ++e)
    if (col[e] < 0 || col[e] >= n) return set_error(MLMQ_ERR_INVALID_ARG, "col[%lld] out of range", (long long)e);
  return MLMQ_OK;
}

static void compute_features(int32_t n, int64_t m, const int32_t* off, const uint32_t* w, mlmq_features* f,
                             uint64_t* deg_hist) {
  double sd = 0, sd2 = 0, maxd = 0;
  for (int i = 0; i < 33; ++i) deg_hist[i] = 0;
  for (int32_t u = 0; u < n; ++u) {
    const double d = (double)(off[u + 1] - off[u]);
    sd += d;
    sd2 += d * d;
    maxd = std::max(maxd, d);
    const uint32_t du = (uint32_t)(off[u + 1] - off[u]);
    deg_hist[du ? 32 - __builtin_clz(du) : 0] += 1;  // bucket k holds degrees in [2^(k-1), 2^k)
  }
  double sw = 0, sw2 = 0, maxw = 0;
  for (int64_t e = 0; e < m; ++e) {
    const double x = (double)w[e];
    sw += x;
    sw2 += x * x;
    maxw = std::max(maxw, x);
  }
  f->n = (double)n;
  f->nnz = (double)m;
  f->avg_deg = sd / n;
  f->max_deg = maxd;
  f->std_deg = std::sqrt(std::max(0.0, sd2 / n - f->avg_deg * f->avg_deg));
  f->avg_w = m ? sw / (double)m : 0;
  f->std_w = m ? std::sqrt(std::max(0.0, sw2 / (double)m - f->avg_w * f->avg_w)) : 0;
  f->max_w = maxw;
}

uint64_t count_degree_above(const mlmq_graph* g, uint32_t th) {
  // vertices with degree > th, bounded above by the histogram buckets that can hold them
  uint64_t c = 0;
  for (int k = 0; k < 33; ++k) {
    const uint64_t hi = k == 0 ? 0 : ((1ull << k) - 1);  // largest degree in bucket k
    if (hi > th) c += g->deg_hist[k];
  }
  return c;
}

}  // namespace mlmq

// ------------------------------------------------------------ C ABI: misc

extern "C" const char* mlmq_last_error(void) { return g_last_error.c_str(); }

extern "C" int mlmq_config_default(mlmq_config* cfg) {
  if (!cfg) return set_error(MLMQ_ERR_INVALID_ARG, "config is NULL");
  if (cfg->struct_size != sizeof(mlmq_config))
    return set_error(MLMQ_ERR_INVALID_ARG, "config struct_size %u != %zu", cfg->struct_size, sizeof(mlmq_config));
  default_config(cfg);
  return MLMQ_OK;
}

extern "C" int mlmq_features_host(int32_t n, int64_t m, const int32_t* row_offsets, const int32_t* col,
                                  const uint32_t* w, mlmq_features* out) {
  if (!out) return set_error(MLMQ_ERR_INVALID_ARG, "out is NULL");
  int rc = validate_csr(n, m, row_offsets, col);
  if (rc) return rc;
  if (m > 0 && !w) return set_error(MLMQ_ERR_INVALID_ARG, "w is NULL");
  uint64_t hist[33];
  compute_features(n, m, row_offsets, w, out, hist);
  return MLMQ_OK;
}

namespace {

void free_graph_arrays(mlmq_graph* g) {
  (void)hipFree(g->d_off);
  (void)hipFree(g->d_adj);
  (void)hipFree(g->d_off_ord);
  (void)hipFree(g->d_adj_ord);
  (void)hipFree(g->d_ord_of);
  g->d_off = g->d_off_ord = nullptr;
  g->d_adj = g->d_adj_ord = nullptr;
  g->d_ord_of = nullptr;
}

// The degree-ordered copy: new ids by decreasing degree (ties by old id),
// rows in new-id order with their edges in the original order.
hipError_t upload_degree_order(mlmq_graph* g, const int32_t* off, const int32_t* col, const uint32_t* w) {
  const int32_t n = g->n;
  const int64_t m = g->m;
  std::vector<uint32_t> order((size_t)n);
  for (int32_t v = 0; v < n; ++v) order[v] = (uint32_t)v;
  std::stable_sort(order.begin(), order.end(),
                   [off](uint32_t a, uint32_t b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
  g->h_ord_of.assign((size_t)n, 0u);
  for (int32_t k = 0; k < n; ++k) g->h_ord_of[order[k]] = (uint32_t)k;
  std::vector<int32_t> off2((size_t)n + 1);
  off2[0] = 0;
  for (int32_t k = 0; k < n; ++k) off2[k + 1] = off2[k] + (off[order[k] + 1] - off[order[k]]);
  std::vector<uint64_t> adj2((size_t)m);
  for (int32_t k = 0; k < n; ++k) {
    const int32_t v = (int32_t)order[k];
    uint64_t* dst = adj2.data() + off2[k];
    for (int32_t e = off[v]; e < off[v + 1]; ++e) *dst++ = g->h_ord_of[col[e]] | ((uint64_t)w[e] << 32);
  }
  hipError_t e = hipMalloc(&g->d_off_ord, sizeof(int32_t) * ((size_t)n + 1));
  if (e == hipSuccess) e = hipMalloc(&g->d_adj_ord, sizeof(uint64_t) * (size_t)m);
  if (e == hipSuccess) e = hipMalloc(&g->d_ord_of, sizeof(uint32_t) * (size_t)n);
  if (e == hipSuccess) e = hipMemcpy(g->d_off_ord, off2.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g->d_adj_ord, adj2.data(), sizeof(uint64_t) * m, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g->d_ord_of, g->h_ord_of.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice);
  return e;
}

}  // namespace

extern "C" int mlmq_graph_create(int32_t n, int64_t m, const int32_t* row_offsets, const int32_t* col,
                                 const uint32_t* w, uint32_t flags, mlmq_graph** out) {
  if (!out) return set_error(MLMQ_ERR_INVALID_ARG, "out is NULL");
  if (flags & ~(MLMQ_MEM_DEVICE | MLMQ_GRAPH_KEEP_ORDER | MLMQ_GRAPH_DEGREE_ORDER))
    return set_error(MLMQ_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  if ((flags & MLMQ_GRAPH_KEEP_ORDER) && (flags & MLMQ_GRAPH_DEGREE_ORDER))
    return set_error(MLMQ_ERR_INVALID_ARG, "MLMQ_GRAPH_KEEP_ORDER and MLMQ_GRAPH_DEGREE_ORDER both set");
  int rc = need_device();
  if (rc) return rc;
  if (n < 1) return set_error(MLMQ_ERR_INVALID_ARG, "n must be >= 1");
  if (m < 0 || m >= (1ll << 31)) return set_error(MLMQ_ERR_INVALID_ARG, "m must be in [0, 2^31)");
  if (!row_offsets || (m > 0 && (!col || !w))) return set_error(MLMQ_ERR_INVALID_ARG, "CSR pointer is NULL");
  // Host copies (validation, features, interleaving col|w into one 8-byte edge).
  std::vector<int32_t> h_off;
  std::vector<int32_t> h_col_buf;
  std::vector<uint32_t> h_w_buf;
  const int32_t* hoff = row_offsets;
  const int32_t* hcol = col;
  const uint32_t* hw = w;
  if (flags & MLMQ_MEM_DEVICE) {
    h_off.resize((size_t)n + 1);
    h_col_buf.resize((size_t)m);
    h_w_buf.resize((size_t)m);
    hipError_t e = hipMemcpy(h_off.data(), row_offsets, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess && m) e = hipMemcpy(h_col_buf.data(), col, sizeof(int32_t) * m, hipMemcpyDeviceToHost);
    if (e == hipSuccess && m) e = hipMemcpy(h_w_buf.data(), w, sizeof(uint32_t) * m, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading device CSR");
    hoff = h_off.data();
    hcol = h_col_buf.data();
    hw = h_w_buf.data();
  }
  rc = validate_csr(n, m, hoff, hcol);
  if (rc) return rc;
  std::unique_ptr<mlmq_graph> g(new mlmq_graph());
  g->n = n;
  g->m = m;
  compute_features(n, m, hoff, hw, &g->features, g->deg_hist);
  uint32_t maxw = 0, minw = kInf;
  for (int64_t e = 0; e < m; ++e) {
    maxw = std::max(maxw, hw[e]);
    minw = std::min(minw, hw[e]);
  }
  g->max_w = maxw;
  g->min_w = m ? minw : 1u;
  g->overflow_safe = (uint64_t)(n - 1) * (uint64_t)maxw < (uint64_t)kInf;
  g->sel_template = selector_pick(g->features);
  std::vector<uint64_t> adj((size_t)m);
  for (int64_t e = 0; e < m; ++e) adj[e] = (uint32_t)hcol[e] | ((uint64_t)hw[e] << 32);
  hipError_t e = hipMalloc(&g->d_off, sizeof(int32_t) * ((size_t)n + 1));
  if (e == hipSuccess) e = hipMalloc(&g->d_adj, sizeof(uint64_t) * std::max<int64_t>(m, 1));
  if (e == hipSuccess) e = hipMemcpy(g->d_off, hoff, sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && m) e = hipMemcpy(g->d_adj, adj.data(), sizeof(uint64_t) * m, hipMemcpyHostToDevice);
  // degree order pays once the labels outgrow the caches (RMAT-23 -5%,
  // RMAT-22 -3.5%, RMAT-20 +6% in plain-solve time)
  const bool skewed = g->features.max_deg >= 16.0 * std::max(1.0, g->features.avg_deg);
  const bool order = (flags & MLMQ_GRAPH_DEGREE_ORDER) || (!(flags & MLMQ_GRAPH_KEEP_ORDER) && skewed && n >= (1 << 22));
  if (e == hipSuccess && order && m > 0) {
    adj.clear();
    adj.shrink_to_fit();
    e = upload_degree_order(g.get(), hoff, hcol, hw);
  }
  if (e != hipSuccess) {
    free_graph_arrays(g.get());
    return hip_fail(e, "uploading graph");
  }
  *out = g.release();
  return MLMQ_OK;
}

extern "C" void mlmq_graph_destroy(mlmq_graph* g) {
  if (!g) return;
  free_graph_arrays(g);
  delete g;
}

extern "C" int mlmq_graph_config(const mlmq_graph* g, mlmq_config* out) {
  if (!g || !out) return set_error(MLMQ_ERR_INVALID_ARG, "NULL argument");
  if (out->struct_size != sizeof(mlmq_config))
    return set_error(MLMQ_ERR_INVALID_ARG, "config struct_size %u != %zu", out->struct_size, sizeof(mlmq_config));
  mlmq_config tmp;
  *out = *resolve_config(g, nullptr, &tmp);
  out->stream = nullptr;
  out->stats_out = nullptr;
  return MLMQ_OK;
}

extern "C" int mlmq_graph_info(const mlmq_graph* g, int32_t* n, int64_t* m, mlmq_features* f) {
  if (!g) return set_error(MLMQ_ERR_INVALID_ARG, "graph is NULL");
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (f) *f = g->features;
  return MLMQ_OK;
}

// ------------------------------------------------------------ planning and memory

namespace mlmq {

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Queue memory of one query for a config.
QueryPlan plan_query(const mlmq_graph* g, const mlmq_config& c, uint32_t extra_nb_log2, uint32_t hub_scale) {
  QueryPlan p;
  const bool pq = c.l2_type == MLMQ_L2_PQ;
  p.nrings = c.l2_type == MLMQ_L2_BUCKET ? c.bmax : (pq ? c.pnum : 1);
  uint64_t cap = c.l2_capacity;
  if (!cap) {
    // FIFO: room for every vertex twice; buckets: a quarter of the vertices
    // per ring (live elements concentrate in a few buckets at a time);
    // priority queues: every vertex twice over all of them.
    cap = c.l2_type == MLMQ_L2_BUCKET ? std::max<uint64_t>(g->n / 4, 1u << 14) : 2ull * g->n;
    cap = std::max<uint64_t>(cap, 1u << 16);
    if (pq) cap = std::max<uint64_t>(cap / p.nrings, 1u << 12);
  } else if (c.l2_type == MLMQ_L2_BUCKET || pq) {
    cap = std::max<uint64_t>(cap / p.nrings, 64);
  }
  // rings: 2^nb_log2 blocks; heaps: node 0 (partial buffer) + 2^nb_log2 - 1 tree nodes
  p.nb_log2 = log2_ceil((cap + 63) / 64 + (pq ? 1 : 0)) + extra_nb_log2;
  // Bucket rings fill with partly filled blocks (the head bucket and those past
  // the write-combining window are written at once, a few elements a block),
  // so on large graphs they get four times the blocks their element count
  // needs, eight times from 4M vertices (a power-law graph of 8M vertices
  // with a near-far or filter L1 over 64-wide buckets peaks at two to four
  // times; the 8M-vertex plan takes 32 rings x 2^18 blocks, 4.3 GB).
  if (c.l2_type == MLMQ_L2_BUCKET && !c.l2_capacity && g->n >= (1 << 20)) p.nb_log2 += g->n >= (1 << 22) ? 3 : 2;
  p.nb_log2 = std::max<uint32_t>(p.nb_log2, 4);
  uint64_t hubs = c.th_hub ? count_degree_above(g, c.th_hub) : 0;
  p.hub_cap = c.th_hub ? (uint32_t)std::min<uint64_t>(std::max<uint64_t>(1024, 4 * hubs) * hub_scale, 1u << 26) : 1;
  const uint64_t nh = (uint64_t)p.nrings << p.nb_log2;
  size_t off = 0;
  p.off_ctrl = off;
  off = align_up(off + sizeof(QueryCtrl), 256);
  p.off_rings = off;
  off = align_up(off + sizeof(RingCtr) * p.nrings, 256);
  p.off_hdr = off;
  off = align_up(off + 8 * nh, 256);
  p.off_data = off;
  off = align_up(off + 512 * nh, 256);
  p.off_hub_rec = off;
  off = align_up(off + 16ull * p.hub_cap, 256);
  p.off_hub_cur = off;
  off = align_up(off + 4ull * p.hub_cap, 256);
  p.off_hub_pub = off;
  off = align_up(off + 4ull * p.hub_cap, 256);
  p.bytes = off;
  p.init_words = (uint32_t)std::max<uint64_t>({(uint64_t)g->n, nh, (uint64_t)p.hub_cap, sizeof(QueryCtrl) / 4});
  return p;
}

QueryDesc make_desc(const mlmq_graph* g, const mlmq_config& c, const QueryPlan& p, char* base, uint32_t* dist,
                    uint32_t source, uint32_t want_wgs) {
  QueryDesc d;
  std::memset(&d, 0, sizeof(d));
  d.off = g->d_off;
  d.adj = g->d_adj;
  d.dist = dist;
  d.ctrl = reinterpret_cast<QueryCtrl*>(base + p.off_ctrl);
  d.rings = reinterpret_cast<RingCtr*>(base + p.off_rings);
  d.hdr = reinterpret_cast<uint64_t*>(base + p.off_hdr);
  d.data = reinterpret_cast<uint64_t*>(base + p.off_data);
  d.hub_rec = reinterpret_cast<uint64_t*>(base + p.off_hub_rec);
  d.hub_cur = reinterpret_cast<uint32_t*>(base + p.off_hub_cur);
  d.hub_pub = reinterpret_cast<uint32_t*>(base + p.off_hub_pub);
  d.n = (uint32_t)g->n;
  d.source = source;
  d.nb_log2 = p.nb_log2;
  d.nrings = p.nrings;
  d.hub_cap = p.hub_cap;
  d.l0_cap = 64u * c.l0_rows;
  d.l1_type = c.l1_type;
  d.l2_type = c.l2_type;
  d.l1_cap = c.l1_type == MLMQ_L1_NONE ? 64u : c.l1_cap;
  d.l1_wb = c.l1_flush_wb;
  d.delta1 = c.delta1;
  d.d2_log2 = c.delta2_log2;
  d.bnum = c.l2_type == MLMQ_L2_BUCKET ? c.bnum : 1;
  d.th_v = c.th_v;
  d.th_hub = c.th_hub;
  d.hub_chunk = c.hub_chunk;
  d.want_wgs = want_wgs;
  d.relax_mode = c.relax_mode;
  // donation threshold: larger graphs carry larger frontiers per wave, and
  // handing work out early only adds global-queue round trips (grid2048:
  // 64 → 20.0 ms vs 22.0 ms with 32; grid512 and grid1024 best at 32)
  d.donate_min = c.donate_min ? c.donate_min : (g->n >= (1 << 21) ? 64u : 32u);
  return d;
}

// Device-memory pool: slabs are kept and reused by later calls.
struct Pool {
  std::mutex mu;
  std::vector<Slab*> free_list;
  ~Pool() {
    for (Slab* s : free_list) {
      (void)hipFree(s->dev);
      (void)hipHostFree(s->host);
      delete s;
    }
  }
};
static Pool& pool() {
  static Pool* p = new Pool();  // never destroyed: the HIP runtime may be gone at exit
  return *p;
}

int slab_acquire(size_t dev_bytes, size_t host_bytes, Slab** out) {
  {
    std::lock_guard<std::mutex> lk(pool().mu);
    auto& fl = pool().free_list;
    Slab* best = nullptr;
    size_t bi = 0;
    for (size_t i = 0; i < fl.size(); ++i)
      if (fl[i]->dev_bytes >= dev_bytes && fl[i]->host_bytes >= host_bytes &&
          (!best || fl[i]->dev_bytes < best->dev_bytes)) {
        best = fl[i];
        bi = i;
      }
    if (best) {
      fl.erase(fl.begin() + bi);
      *out = best;
      return MLMQ_OK;
    }
  }
  Slab* s = new Slab();
  s->dev_bytes = align_up(dev_bytes, 1 << 20);
  s->host_bytes = align_up(std::max<size_t>(host_bytes, 4096), 4096);
  hipError_t e = hipMalloc(&s->dev, s->dev_bytes);
  if (e == hipSuccess) e = hipHostMalloc(&s->host, s->host_bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(s->dev);
    delete s;
    // Give cached slabs back to the device and try once more.
    std::vector<Slab*> drop;
    {
      std::lock_guard<std::mutex> lk(pool().mu);
      drop.swap(pool().free_list);
    }
    for (Slab* d : drop) {
      (void)hipFree(d->dev);
      (void)hipHostFree(d->host);
      delete d;
    }
    s = new Slab();
    s->dev_bytes = align_up(dev_bytes, 1 << 20);
    s->host_bytes = align_up(std::max<size_t>(host_bytes, 4096), 4096);
    e = hipMalloc(&s->dev, s->dev_bytes);
    if (e == hipSuccess) e = hipHostMalloc(&s->host, s->host_bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      (void)hipFree(s->dev);
      delete s;
      return hip_fail(e, "allocating queue memory");
    }
  }
  *out = s;
  return MLMQ_OK;
}

void slab_release(Slab* s) {
  if (!s) return;
  std::lock_guard<std::mutex> lk(pool().mu);
  pool().free_list.push_back(s);
}

void pool_trim() {
  std::vector<Slab*> drop;
  {
    std::lock_guard<std::mutex> lk(pool().mu);
    drop.swap(pool().free_list);
  }
  for (Slab* d : drop) {
    if (d->graph_exec) (void)hipGraphExecDestroy(d->graph_exec);
    (void)hipFree(d->dev);
    (void)hipHostFree(d->host);
    delete d;
  }
}

// Launch shape for a config: workgroup size, LDS bytes and the number of
// persistent workgroups that fit on the device at once.
int launch_shape(const mlmq_config& c, uint32_t l1_cap, bool two, bool stage, bool pq, LaunchShape* out) {
  const DeviceInfo* di = device_info();
  LaunchShape s;
  s.wg = c.wg_size;
  s.waves = c.wg_size / 64;
  s.l1_cap = l1_cap;
  s.two = two;
  s.stage = stage;
  s.pq = pq;
  s.lds = worker_lds_bytes(s.waves, l1_cap, two, stage);
  if (s.lds > di->lds_per_wg)
    return set_error(MLMQ_ERR_INVALID_ARG, "L1 needs %zu bytes of LDS per workgroup (limit %zu)", s.lds,
                     di->lds_per_wg);
  int per_cu = 0;
  hipError_t e = worker_occupancy(s.wg, s.lds, s.pq, &per_cu);
  if (e != hipSuccess) return hip_fail(e, "occupancy query");
  if (per_cu < 1) return set_error(MLMQ_ERR_INVALID_ARG, "workgroup shape does not fit on a CU");
  s.max_grid = (uint32_t)per_cu * (uint32_t)di->cus;
  s.grid = c.grid_wgs ? std::min(c.grid_wgs, s.max_grid) : s.max_grid;
  *out = s;
  return MLMQ_OK;
}

LaunchArgs make_args(const QueryDesc* d_desc, BatchCtrl* d_batch, int nq, const LaunchShape& s, uint32_t timeout_ms,
                     uint32_t* d_beats) {
  const DeviceInfo* di = device_info();
  LaunchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.queries = d_desc;
  a.batch = d_batch;
  a.nq = nq;
  a.l1_cap = s.l1_cap;
  a.l1_two = s.two ? 1u : 0u;
  a.stage = s.stage ? 1u : 0u;
  a.waves = s.waves;
  a.pq = s.pq ? 1u : 0u;
  a.timeout_ticks = (uint64_t)(timeout_ms ? timeout_ms : 60000) * di->ticks_per_ms;
  a.cap_wait_ticks = 20ull * di->ticks_per_ms;
  a.beats = d_beats;
  return a;
}

static bool is_device_ptr(const void* p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

// Queue counters of a finished (or stopped) query, for error messages.
std::string describe_query_state(const QueryDesc& d, const uint32_t* d_beats, uint32_t nbeats) {
  QueryCtrl hc;
  std::vector<RingCtr> hr(d.nrings);
  if (hipMemcpy(&hc, d.ctrl, sizeof(hc), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hr.data(), d.rings, sizeof(RingCtr) * d.nrings, hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return "queue state unreadable";
  }
  uint64_t reserved = hc.hub_units.v;
  if (d.l2_type == MLMQ_L2_PQ)
    reserved += hc.pq_in.v;  // elements written to the priority queues
  else
    for (const RingCtr& r : hr) reserved += r.tail.v;
  char buf[256];
  snprintf(buf, sizeof(buf), "done %u reserved %llu cur %u hungry %u active %u hub %u/%u; tail/head:", hc.done.v,
           (unsigned long long)reserved, hc.cur.v, hc.hungry.v, hc.active.v, hc.hub_head.v, hc.hub_tail.v);
  std::string out = buf;
  for (uint32_t i = 0; i < d.nrings && i < 64; ++i) {
    if (!hr[i].tail.v && !hr[i].head.v) continue;
    snprintf(buf, sizeof(buf), " r%u=%u/%u", i, hr[i].tail.v, hr[i].head.v);
    out += buf;
  }
  if (d_beats && nbeats) {
    std::vector<uint32_t> hb(nbeats);
    if (hipMemcpy(hb.data(), d_beats, 4ull * nbeats, hipMemcpyDeviceToHost) == hipSuccess) {
      uint32_t hist[16] = {0};
      for (uint32_t b : hb) hist[(b >> 24) & 15u] += 1;
      out += "; waves by last program point:";
      for (int p = 0; p < 16; ++p)
        if (hist[p]) {
          snprintf(buf, sizeof(buf), " p%d=%u", p, hist[p]);
          out += buf;
        }
    }
  }
  return out;
}

int status_to_code(uint32_t st) {
  switch (st) {
    case kStOk:
      return MLMQ_OK;
    case kStCapacity:
    case kStHubCapacity:
      return MLMQ_ERR_QUEUE_CAPACITY;
    case kStTimeout:
      return MLMQ_ERR_TIMEOUT;
    case kStCanceled:
      return MLMQ_ERR_CANCELED;
    default:
      return MLMQ_ERR_DEVICE;
  }
}

void fill_stats(mlmq_stats* st, const QueryCtrl& h, double ms, double worker_ms, uint32_t grid, uint32_t retries) {
  if (!st) return;
  const uint32_t sz = st->struct_size;
  std::memset(st, 0, sizeof(*st));
  st->struct_size = sz;
  st->status = h.error.v;
  st->kernel_ms = ms;
  st->worker_ms = worker_ms;
  st->expansions = h.stats[kCtExpansions];
  st->stale = h.stats[kCtStale];
  st->edges = h.stats[kCtEdges];
  st->pushes = h.stats[kCtPushes];
  st->l1_writes = h.stats[kCtL1Writes];
  st->l1_reads = h.stats[kCtL1Reads];
  st->l2_writes = h.stats[kCtL2Writes];
  st->l2_reads = h.stats[kCtL2Reads];
  st->hub_chunks = h.stats[kCtHubChunks];
  st->flushes = h.stats[kCtFlushes];
  st->donations = h.stats[kCtDonations];
  st->atomics = h.stats[kCtAtomics];
  st->wave_ms = (double)h.stats[kCtWaveTicks] / (double)device_info()->ticks_per_ms;
  st->idle_ms = (double)h.stats[kCtIdleTicks] / (double)device_info()->ticks_per_ms;
  st->grid_wgs = grid;
  st->retries = retries;
}

// Wait for the stream with a host-side watchdog: if the device does not
// finish within timeout_ms + grace, snapshot its queue counters and per-wave
// heartbeats (read through a side stream, so the reads do not queue behind the
// kernel), raise the device cancel flag and wait once more. Returns
// hipSuccess, a HIP error, or hipErrorLaunchTimeOut when the kernel would not
// stop (its memory must then be left alone); the snapshot goes to the error
// message.
hipError_t wait_with_watchdog(hipStream_t stream, uint32_t timeout_ms, uint32_t* d_cancel, uint32_t* h_one,
                              const WatchdogView& view, hipStream_t side) {
  using clk = std::chrono::steady_clock;
  const auto limit = clk::now() + std::chrono::milliseconds((timeout_ms ? timeout_ms : 60000) + 3000);
  for (;;) {
    hipError_t e = hipStreamQuery(stream);
    if (e != hipErrorNotReady) return e;
    if (clk::now() > limit) break;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  if (!side) {
    static hipStream_t own = nullptr;
    static std::once_flag once;
    std::call_once(once, [] { (void)hipStreamCreateWithFlags(&own, hipStreamNonBlocking); });
    side = own;
  }
  std::string snap = "watchdog snapshot:";
  if (view.d_ctrl) {
    uint32_t* hb = nullptr;
    const size_t bytes = sizeof(QueryCtrl) + sizeof(RingCtr) + 4ull * view.nbeats;
    if (hipHostMalloc(reinterpret_cast<void**>(&hb), bytes, hipHostMallocDefault) == hipSuccess) {
      QueryCtrl* hc = reinterpret_cast<QueryCtrl*>(hb);
      RingCtr* hr = reinterpret_cast<RingCtr*>(hc + 1);
      uint32_t* beats = reinterpret_cast<uint32_t*>(hr + 1);
      hipError_t e = hipMemcpyAsync(hc, view.d_ctrl, sizeof(QueryCtrl), hipMemcpyDeviceToHost, side);
      if (e == hipSuccess) e = hipMemcpyAsync(hr, view.d_rings, sizeof(RingCtr), hipMemcpyDeviceToHost, side);
      if (e == hipSuccess && view.nbeats)
        e = hipMemcpyAsync(beats, view.d_beats, 4ull * view.nbeats, hipMemcpyDeviceToHost, side);
      const auto lim = clk::now() + std::chrono::milliseconds(2000);
      while (e == hipSuccess && hipStreamQuery(side) == hipErrorNotReady && clk::now() < lim)
        std::this_thread::sleep_for(std::chrono::microseconds(200));
      if (e == hipSuccess && hipStreamQuery(side) == hipSuccess) {
        char buf[256];
        snprintf(buf, sizeof(buf), " done=%u tail0=%u head0=%u terminate=%u error=%u joined=%u finished=%u;",
                 hc->done.v, hr->tail.v, hr->head.v, hc->terminate.v, hc->error.v, hc->joined.v, hc->finished.v);
        snap += buf;
        uint32_t hist[16] = {0};
        for (uint32_t i = 0; i < view.nbeats; ++i) hist[(beats[i] >> 24) & 15u] += 1;
        snap += " waves by program point:";
        for (int p = 0; p < 16; ++p)
          if (hist[p]) {
            snprintf(buf, sizeof(buf), " p%d=%u", p, hist[p]);
            snap += buf;
          }
      } else {
        snap += " (device memory could not be read)";
      }
      (void)hipHostFree(hb);
    }
  }
  g_last_error = snap;
  *h_one = 1;
  (void)hipMemcpyAsync(d_cancel, h_one, 4, hipMemcpyHostToDevice, side);
  const auto limit2 = clk::now() + std::chrono::milliseconds(5000);
  for (;;) {
    hipError_t e = hipStreamQuery(stream);
    if (e != hipErrorNotReady) return e == hipSuccess ? hipErrorLaunchTimeOut : e;
    if (clk::now() > limit2) return hipErrorLaunchTimeOut;
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
}

const mlmq_config* resolve_config(const mlmq_graph* g, const mlmq_config* cfg, mlmq_config* tmp) {
  if (cfg) return cfg;
  std::lock_guard<std::mutex> lk(const_cast<mlmq_graph*>(g)->mu);
  if (g->has_tuned) {
    *tmp = g->tuned;
  } else if (g->sel_template < 0 || template_config(g, g->sel_template, tmp) != MLMQ_OK) {
    tmp->struct_size = sizeof(mlmq_config);
    default_config(tmp);
    heuristic_config(g, tmp);
  }
  return tmp;
}

// Defaults seeded from the Table 2 features (Section 3.5's heuristics):
// mesh/road-like graphs keep a FIFO L2 with local L0/L1 queues; skewed
// power-law graphs get buckets and the grid-wide hub tier.
void heuristic_config(const mlmq_graph* g, mlmq_config* c) {
  // Feature-driven defaults (Section 3.5, Table 2 features), set from
  // measurements on the synthetic stand-ins of the paper's graph classes.
  const mlmq_features& f = g->features;
  const uint32_t mean_w = (uint32_t)std::max(1.0, f.avg_w);
  c->delta2_log2 = log2_ceil(std::max<uint32_t>(1, mean_w));
  uint32_t num = 1, den = 1;  // share of the resident waves to launch
  if (f.max_deg > 64 && f.std_deg > f.avg_deg) {
    // power-law: near-far L1 with a narrow window over a FIFO L2, hub chunks
    // for the top vertices. A small L1 sends work to L2 early, where idle
    // waves find it (a large one keeps long private chains, which makes small
    // graphs latency-bound); the launch grows with the edge count up to six
    // one-wave workgroups per CU.
    c->l0_rows = 1;
    c->l1_type = MLMQ_L1_NEARFAR;
    c->l2_type = MLMQ_L2_FIFO;
    c->delta1 = std::max<uint32_t>(1, mean_w / 2);
    const double m = f.nnz;
    c->th_hub = m < 64e6 ? 8192 : 16384;
    c->hub_chunk = 4096;
    c->l1_cap = m < 64e6 ? 128 : 256;
    const uint32_t cus = (uint32_t)std::max(1, device_info()->cus);
    c->grid_wgs = (uint32_t)std::min<double>(6.0 * cus, std::max(512.0, m / 32768.0));
    return;
  } else {
    // low, even degree (meshes, road-like grids): no L0 (it would follow
    // private chains ahead of the frontier), near-far L1 two mean weights
    // wide, FIFO L2 with donations, two ninths of the resident waves, and
    // atomicMin without the label pre-check (the solve is latency-bound: one
    // round trip less per hop matters more than the extra atomics)
    c->l0_rows = 0;
    c->relax_mode = MLMQ_RELAX_ATOMIC;
    c->l1_type = MLMQ_L1_NEARFAR;
    c->l2_type = MLMQ_L2_FIFO;
    c->delta1 = std::max<uint32_t>(1, mean_w * 2);
    c->th_hub = 0;
    num = 2;
    den = 9;
  }
  LaunchShape s;
  if (num != den && launch_shape(*c, c->l1_cap, c->l1_type == MLMQ_L1_NEARFAR, c->l2_type == MLMQ_L2_BUCKET,
                                c->l2_type == MLMQ_L2_PQ, &s) ==
                        MLMQ_OK)
    c->grid_wgs = std::max<uint32_t>(64, s.max_grid * num / den);
  else
    (void)hipGetLastError();
}

// One solve attempt sequence (with capacity retries) on a slab.
int run_single(const mlmq_graph* g, uint32_t source, uint32_t* dist_out, const mlmq_config& c, bool unit_weights) {
  int rc = check_config(&c);
  if (rc) return rc;
  hipStream_t stream = reinterpret_cast<hipStream_t>(c.stream);
  const bool dev_out = is_device_ptr(dist_out);
  // power-law graphs are solved on their degree-ordered copy, whose labels
  // are gathered back into the caller's order at the end
  const bool ordered = g->d_ord_of != nullptr;
  LaunchShape shape;
  rc = launch_shape(c, c.l1_type == MLMQ_L1_NONE ? 64u : c.l1_cap, c.l1_type == MLMQ_L1_NEARFAR,
                    c.l2_type == MLMQ_L2_BUCKET, c.l2_type == MLMQ_L2_PQ, &shape);
  if (rc) return rc;
  uint32_t extra = 0, hub_scale = 1, retries = 0;
  for (;;) {
    QueryPlan p = plan_query(g, c, extra, hub_scale);
    const size_t desc_off = align_up(p.bytes, 256);
    const size_t batch_off = align_up(desc_off + sizeof(QueryDesc), 256);
    const size_t beats_off = align_up(batch_off + sizeof(BatchCtrl), 256);
    const size_t dist_off = align_up(beats_off + 4ull * shape.grid, 256);
    // the solve's own labels (unless it writes the caller's device buffer),
    // then, for a host buffer after an ordered solve, the gathered copy
    const size_t out_off = align_up(dist_off + (dev_out && !ordered ? 0 : 4ull * g->n), 256);
    const size_t dev_bytes = out_off + (!dev_out && ordered ? 4ull * g->n : 0);
    const size_t host_bytes = sizeof(QueryCtrl) + sizeof(QueryDesc) + 64;
    Slab* slab = nullptr;
    rc = slab_acquire(dev_bytes, host_bytes, &slab);
    if (rc) return rc;
    char* base = static_cast<char*>(slab->dev);
    uint32_t* d_dist = dev_out && !ordered ? dist_out : reinterpret_cast<uint32_t*>(base + dist_off);
    uint32_t* d_final = dev_out ? dist_out : (ordered ? reinterpret_cast<uint32_t*>(base + out_off) : d_dist);
    QueryDesc* d_desc = reinterpret_cast<QueryDesc*>(base + desc_off);
    BatchCtrl* d_batch = reinterpret_cast<BatchCtrl*>(base + batch_off);
    QueryCtrl* h_ctrl = reinterpret_cast<QueryCtrl*>(slab->host);
    QueryDesc* h_desc = reinterpret_cast<QueryDesc*>(static_cast<char*>(slab->host) + sizeof(QueryCtrl));
    *h_desc = make_desc(g, c, p, base, d_dist, source, shape.grid);
    if (ordered) {
      h_desc->off = g->d_off_ord;
      h_desc->adj = g->d_adj_ord;
      h_desc->source = g->h_ord_of[source];
    }
    h_desc->unit_w = unit_weights ? 1u : 0u;
    // breadth-first levels: early hand-out pays (grid2048 17.4 vs 19.4 ms)
    if (unit_weights && !c.donate_min) h_desc->donate_min = 32u;
    uint32_t* d_beats = reinterpret_cast<uint32_t*>(base + beats_off);
    LaunchArgs a = make_args(d_desc, d_batch, 1, shape, c.timeout_ms, d_beats);
    hipEvent_t ev0 = nullptr, evw = nullptr, ev1 = nullptr;
    hipError_t e = hipSuccess;
    if (c.stats_out) {
      e = hipEventCreate(&ev0);
      if (e == hipSuccess) e = hipEventCreate(&evw);
      if (e == hipSuccess) e = hipEventCreate(&ev1);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(d_desc, h_desc, sizeof(QueryDesc), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && ev0) e = hipEventRecord(ev0, stream);
    if (e == hipSuccess) e = launch_init(d_desc, d_batch, 1, p.init_words, stream);
    if (e == hipSuccess && evw) e = hipEventRecord(evw, stream);
    if (e == hipSuccess) e = launch_worker(a, shape.grid, shape.wg, shape.lds, stream);
    if (e == hipSuccess && ev1) e = hipEventRecord(ev1, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h_ctrl, base + p.off_ctrl, sizeof(QueryCtrl), hipMemcpyDeviceToHost, stream);
    uint32_t* h_one = reinterpret_cast<uint32_t*>(h_desc + 1) + 1;
    WatchdogView view;
    view.d_ctrl = reinterpret_cast<const QueryCtrl*>(base + p.off_ctrl);
    view.d_rings = reinterpret_cast<const RingCtr*>(base + p.off_rings);
    view.d_beats = d_beats;
    view.nbeats = shape.grid;
    if (e == hipSuccess) e = wait_with_watchdog(stream, c.timeout_ms, &d_batch->cancel.v, h_one, view);
    if (e == hipErrorLaunchTimeOut) {
      // the kernel overran its watchdog; if it did not stop either, its memory is never reused
      const std::string snap = g_last_error;
      if (hipStreamQuery(stream) == hipSuccess) slab_release(slab);
      return set_error(MLMQ_ERR_TIMEOUT, "device overran its timeout (%s)", snap.c_str());
    }
    float ms = 0, wms = 0;
    if (e == hipSuccess && ev0) e = hipEventElapsedTime(&ms, ev0, ev1);
    if (e == hipSuccess && evw) e = hipEventElapsedTime(&wms, evw, ev1);
    if (ev0) (void)hipEventDestroy(ev0);
    if (evw) (void)hipEventDestroy(evw);
    if (ev1) (void)hipEventDestroy(ev1);
    if (e != hipSuccess) {
      slab_release(slab);
      return hip_fail(e, "solve");
    }
    const uint32_t st = h_ctrl->error.v;
    if ((st == kStCapacity || st == kStHubCapacity) && retries < c.max_retries) {
      slab_release(slab);
      if (st == kStCapacity) extra += 1;
      else hub_scale *= 4;
      ++retries;
      pool_trim();
      continue;
    }
    rc = status_to_code(st);
    if (rc == MLMQ_OK && h_ctrl->overflow.v && !g->overflow_safe) {
      // exact overflow test: an edge from a finite label to an unreachable one
      uint32_t* h_flag = reinterpret_cast<uint32_t*>(h_desc + 1);
      uint32_t* d_flag = &d_batch->cancel.v;
      e = hipMemsetAsync(d_flag, 0, 4, stream);
      if (e == hipSuccess) e = launch_overflow_check(d_desc, d_flag, stream);
      if (e == hipSuccess) e = hipMemcpyAsync(h_flag, d_flag, 4, hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) {
        slab_release(slab);
        return hip_fail(e, "overflow check");
      }
      if (*h_flag) rc = set_error(MLMQ_ERR_DISTANCE_OVERFLOW, "a reachable distance does not fit below 2^32-1");
    } else if (rc != MLMQ_OK) {
      const std::string state = describe_query_state(*h_desc, d_beats, shape.grid);
      set_error(rc, "solve failed with device status %u (%s)", st, state.c_str());
    }
    if (ordered && (rc == MLMQ_OK || rc == MLMQ_ERR_DISTANCE_OVERFLOW)) {
      e = launch_unorder(d_dist, g->d_ord_of, (uint32_t)g->n, d_final, stream);
      if (e == hipSuccess && dev_out) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) rc = hip_fail(e, "gathering distances");
    }
    if (!dev_out && (rc == MLMQ_OK || rc == MLMQ_ERR_DISTANCE_OVERFLOW)) {
      e = hipMemcpyAsync(dist_out, d_final, 4ull * g->n, hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) rc = hip_fail(e, "copying distances");
    }
    fill_stats(c.stats_out, *h_ctrl, ms, wms, shape.grid, retries);
    slab_release(slab);
    return rc;
  }
}

}  // namespace mlmq

// ------------------------------------------------------------ C ABI: solves

extern "C" int mlmq_sssp(const mlmq_graph* g, uint32_t source, uint32_t* dist_out, const mlmq_config* cfg) {
  if (!g) return set_error(MLMQ_ERR_INVALID_ARG, "graph is NULL");
  if (!dist_out) return set_error(MLMQ_ERR_INVALID_ARG, "dist_out is NULL");
  if (source >= (uint32_t)g->n) return set_error(MLMQ_ERR_INVALID_ARG, "source %u >= n %d", source, g->n);
  int rc = need_device();
  if (rc) return rc;
  mlmq_config tmp;
  const mlmq_config* c = resolve_config(g, cfg, &tmp);
  return run_single(g, source, dist_out, *c);
}

namespace {

// Per-device state of the allocation-free solve, set up on its first call on
// a device: the fixed queue array's address and a stream for the watchdog's
// cancel store. Calls on one device hold its lock for the whole solve, since
// they all use the same array.
struct NoAllocDevice {
  std::mutex mu;
  void* scratch = nullptr;
  hipStream_t side = nullptr;
  bool ready = false;
  uint32_t one = 1;
  uint32_t zero = 0;
};

int noalloc_device(int dev, NoAllocDevice** out) {
  static std::mutex mu;
  static NoAllocDevice devs[64];
  if (dev < 0 || dev >= 64) return set_error(MLMQ_ERR_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(mu);
  NoAllocDevice& d = devs[dev];
  if (!d.ready) {
    hipError_t e = noalloc_scratch(dev, &d.scratch);
    if (e != hipSuccess) return hip_fail(e, "address of the fixed queue array");
    e = hipStreamCreateWithFlags(&d.side, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "watchdog stream");
    d.ready = true;
  }
  *out = &d;
  return MLMQ_OK;
}

}  // namespace

extern "C" int mlmq_sssp_noalloc(const mlmq_graph* g, uint32_t source, uint32_t* dist_out, const mlmq_config* cfg) {
  if (!g) return set_error(MLMQ_ERR_INVALID_ARG, "graph is NULL");
  if (!dist_out) return set_error(MLMQ_ERR_INVALID_ARG, "dist_out is NULL");
  if (source >= (uint32_t)g->n) return set_error(MLMQ_ERR_INVALID_ARG, "source %u >= n %d", source, g->n);
  int rc = need_device();
  if (rc) return rc;
  mlmq_config tmp;
  const mlmq_config& c = *resolve_config(g, cfg, &tmp);
  rc = check_config(&c);
  if (rc) return rc;
  if (!is_device_ptr(dist_out)) return set_error(MLMQ_ERR_INVALID_ARG, "dist_out must be device memory");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  NoAllocDevice* nd = nullptr;
  rc = noalloc_device(dev, &nd);
  if (rc) return rc;
  LaunchShape shape;
  rc = launch_shape(c, c.l1_type == MLMQ_L1_NONE ? 64u : c.l1_cap, c.l1_type == MLMQ_L1_NEARFAR,
                    c.l2_type == MLMQ_L2_BUCKET, c.l2_type == MLMQ_L2_PQ, &shape);
  if (rc) return rc;
  // Layout inside the array: queues, descriptor, launch control words, the
  // overflow flag and one heartbeat word per workgroup.
  const QueryPlan p = plan_query(g, c, 0, 1);
  const size_t desc_off = align_up(p.bytes, 256);
  const size_t batch_off = align_up(desc_off + sizeof(QueryDesc), 256);
  const size_t flag_off = align_up(batch_off + sizeof(BatchCtrl), 256);
  const size_t beats_off = align_up(flag_off + 4, 256);
  const size_t total = align_up(beats_off + 4ull * shape.grid, 256);
  if (total > kNoAllocScratchBytes)
    return set_error(MLMQ_ERR_INVALID_ARG,
                     "queue memory of this solve (%zu bytes) exceeds the %zu bytes of the allocation-free entry point",
                     total, kNoAllocScratchBytes);
  hipStream_t stream = reinterpret_cast<hipStream_t>(c.stream);
  std::lock_guard<std::mutex> lk(nd->mu);
  char* base = static_cast<char*>(nd->scratch);
  QueryDesc* d_desc = reinterpret_cast<QueryDesc*>(base + desc_off);
  BatchCtrl* d_batch = reinterpret_cast<BatchCtrl*>(base + batch_off);
  uint32_t* d_flag = reinterpret_cast<uint32_t*>(base + flag_off);
  uint32_t* d_beats = reinterpret_cast<uint32_t*>(base + beats_off);
  const QueryDesc h_desc = make_desc(g, c, p, base, dist_out, source, shape.grid);
  const LaunchArgs a = make_args(d_desc, d_batch, 1, shape, c.timeout_ms, d_beats);
  // The init kernel resets every queue word, counter and control word the
  // worker reads (the array keeps whatever the previous call left).
  e = hipMemcpyAsync(d_desc, &h_desc, sizeof(QueryDesc), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = launch_init(d_desc, d_batch, 1, p.init_words, stream);
  if (e == hipSuccess) e = launch_worker(a, shape.grid, shape.wg, shape.lds, stream);
  WatchdogView view;  // no snapshot: it would allocate pinned memory
  nd->one = 1;
  if (e == hipSuccess) e = wait_with_watchdog(stream, c.timeout_ms, &d_batch->cancel.v, &nd->one, view, nd->side);
  if (e == hipErrorLaunchTimeOut) return set_error(MLMQ_ERR_TIMEOUT, "device overran its timeout");
  QueryCtrl h_ctrl;
  if (e == hipSuccess) e = hipMemcpyAsync(&h_ctrl, h_desc.ctrl, sizeof(QueryCtrl), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "solve");
  const uint32_t st = h_ctrl.error.v;
  rc = status_to_code(st);
  if (rc == MLMQ_OK && h_ctrl.overflow.v && !g->overflow_safe) {
    // exact overflow test, as in mlmq_sssp
    uint32_t h_flag = 0;
    nd->zero = 0;
    e = hipMemcpyAsync(d_flag, &nd->zero, 4, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_overflow_check(d_desc, d_flag, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&h_flag, d_flag, 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "overflow check");
    if (h_flag) rc = set_error(MLMQ_ERR_DISTANCE_OVERFLOW, "a reachable distance does not fit below 2^32-1");
  } else if (rc != MLMQ_OK) {
    set_error(rc, "solve failed with device status %u (no capacity retry without allocation)", st);
  }
  fill_stats(c.stats_out, h_ctrl, 0.0, 0.0, shape.grid, 0);
  return rc;
}

extern "C" int mlmq_latency_probe(const mlmq_graph* g, uint32_t source, uint32_t hops, void* stream,
                                  double* hop_ns_out, double* handoff_ns_out) {
  if (!g || !hop_ns_out || !handoff_ns_out) return set_error(MLMQ_ERR_INVALID_ARG, "NULL argument");
  if (source >= (uint32_t)g->n) return set_error(MLMQ_ERR_INVALID_ARG, "source %u >= n %d", source, g->n);
  if (hops < 1 || hops > (1u << 24)) return set_error(MLMQ_ERR_INVALID_ARG, "hops must be in [1, 2^24]");
  int rc = need_device();
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  constexpr uint32_t kRounds = 2048;
  const size_t lab_bytes = align_up(4ull * g->n, 256);
  void* buf = nullptr;
  hipError_t e = hipMalloc(&buf, lab_bytes + 256 + 64);
  if (e != hipSuccess) return hip_fail(e, "probe scratch");
  auto* lab = static_cast<uint32_t*>(buf);
  auto* word = reinterpret_cast<uint32_t*>(static_cast<char*>(buf) + lab_bytes);
  auto* d_out = reinterpret_cast<uint64_t*>(static_cast<char*>(buf) + lab_bytes + 256);
  uint64_t h_out[4] = {0, 0, 0, 0};
  e = hipMemsetAsync(lab, 0xFF, lab_bytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(word, 0, 256 + 64, s);
  const uint64_t limit = 2000ull * device_info()->ticks_per_ms;  // 2 s
  if (e == hipSuccess)
    e = launch_latency_probes(g->d_off, g->d_adj, lab, (uint32_t)g->n, source, hops, word, kRounds, limit, d_out, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h_out, d_out, sizeof(h_out), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_fail(e, "latency probes");
  if (h_out[3]) return set_error(MLMQ_ERR_TIMEOUT, "hand-off probe: the second workgroup did not answer");
  const double ns_per_tick = 1e6 / (double)device_info()->ticks_per_ms;
  *hop_ns_out = (double)h_out[0] * ns_per_tick / hops;
  *handoff_ns_out = (double)h_out[2] * ns_per_tick / (2.0 * kRounds);
  return MLMQ_OK;
}

extern "C" int mlmq_bfs(const mlmq_graph* g, uint32_t source, uint32_t* levels_out, const mlmq_config* cfg) {
  if (!g) return set_error(MLMQ_ERR_INVALID_ARG, "graph is NULL");
  if (!levels_out) return set_error(MLMQ_ERR_INVALID_ARG, "levels_out is NULL");
  if (source >= (uint32_t)g->n) return set_error(MLMQ_ERR_INVALID_ARG, "source %u >= n %d", source, g->n);
  int rc = need_device();
  if (rc) return rc;
  mlmq_config tmp;
  if (cfg) return run_single(g, source, levels_out, *cfg, true);
  // the graph's config with its weight-dependent windows set for unit steps:
  // the near set of a near-far L1 is the current level
  tmp = *resolve_config(g, nullptr, &tmp);
  tmp.delta1 = 1;
  tmp.delta2_log2 = 0;
  return run_single(g, source, levels_out, tmp, true);
}

extern "C" int mlmq_check(const mlmq_graph* g, uint32_t source, const uint32_t* dist, void* stream,
                          uint64_t* violations_out, float* edge_pass_ms_out) {
  if (!g) return set_error(MLMQ_ERR_INVALID_ARG, "graph is NULL");
  if (!dist) return set_error(MLMQ_ERR_INVALID_ARG, "dist is NULL");
  if (!violations_out) return set_error(MLMQ_ERR_INVALID_ARG, "violations_out is NULL");
  if (source >= (uint32_t)g->n) return set_error(MLMQ_ERR_INVALID_ARG, "source %u >= n %d", source, g->n);
  if (g->min_w == 0)
    return set_error(MLMQ_ERR_INVALID_ARG, "graph has zero-weight edges: the check needs positive weights");
  int rc = need_device();
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t tight_bytes = align_up((size_t)g->n, 256);
  void* buf = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipError_t e = hipMalloc(&buf, tight_bytes + sizeof(unsigned long long));
  if (e != hipSuccess) return hip_fail(e, "check scratch");
  auto* tight = static_cast<uint8_t*>(buf);
  auto* bad = reinterpret_cast<unsigned long long*>(static_cast<char*>(buf) + tight_bytes);
  unsigned long long h_bad = 0;
  float ms = 0.f;
  e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  if (e == hipSuccess) e = hipMemsetAsync(buf, 0, tight_bytes + sizeof(unsigned long long), s);
  if (e == hipSuccess)
    e = launch_check(g->d_off, g->d_adj, dist, (uint32_t)g->n, (uint32_t)g->m, source, tight, bad, ev0, ev1, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&h_bad, bad, sizeof(h_bad), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_fail(e, "optimality check");
  *violations_out = h_bad;
  if (edge_pass_ms_out) *edge_pass_ms_out = ms;
  return MLMQ_OK;
}
