// Input-adaptive configuration (Section 3.5): a fixed list of candidate
// configurations ("templates", each knob relative to the graph's Table 2
// features or to the device), the learned selector -- a random-forest
// regressor that predicts a template's performance relative to the best one
// from the graph features and the template's knobs -- and the autotuner,
// which times the selector's top picks beside the feature-driven default.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/mlmq.h"
#include "mlmq_api_internal.h"
#include "mlmq_internal.h"

using namespace mlmq;

namespace {

// One candidate. delta1 = mean weight * d1m (near-far window / filter step),
// bucket width = the power of two nearest to mean weight * d2m, launch =
// grid * (CUs * 12) one-wave workgroups (12 = three waves on each of a CU's
// four SIMDs, the worker's register budget), capped by what fits.
struct Template {
  uint8_t l0, l1, l2, relax;
  float d1m, d2m;
  uint16_t cap;
  float grid;
  uint16_t donate, wb;
  uint8_t bnum;
  uint16_t thv;
};

constexpr uint8_t N = MLMQ_L1_NONE, V = MLMQ_L1_VEC, NF = MLMQ_L1_NEARFAR, FQ = MLMQ_L1_FILTER, SLF = MLMQ_L1_SLF;
constexpr uint8_t FI = MLMQ_L2_FIFO, DQ = MLMQ_L2_BUCKET;
constexpr uint8_t PRE = MLMQ_RELAX_PRECHECK, AT = MLMQ_RELAX_ATOMIC;

// The search space: every L1 policy over both L2 types, with and without
// register queues, around the two regimes the feature heuristic separates
// (skewed power-law graphs: small private L1, wide launch, label pre-check;
// low even degree: large near-far L1, narrow launch, atomicMin alone), plus
// variants of the spill thresholds (donation size, L1V flush period, whole-
// wave threshold) and the single-global-queue baselines.
//                          l0  l1  l2  relax d1m   d2m  cap   grid   don  wb  bn  thv
const Template kTemplates[] = {
    // near-far over the FIFO ring
    {1, NF, FI, PRE, 0.5f, 1.0f, 128, 0.333f, 32, 64, 4, 32},
    {1, NF, FI, PRE, 0.5f, 1.0f, 256, 0.5f, 64, 64, 4, 32},
    {1, NF, FI, PRE, 0.5f, 1.0f, 128, 0.167f, 32, 64, 4, 32},
    {1, NF, FI, PRE, 2.0f, 1.0f, 256, 0.5f, 32, 64, 4, 32},
    {0, NF, FI, AT, 2.0f, 1.0f, 1024, 0.222f, 32, 64, 4, 32},
    {0, NF, FI, AT, 2.0f, 1.0f, 1024, 0.222f, 64, 64, 4, 32},
    {0, NF, FI, AT, 1.0f, 1.0f, 1024, 0.333f, 32, 64, 4, 32},
    {0, NF, FI, AT, 4.0f, 1.0f, 1024, 0.111f, 32, 64, 4, 32},
    {0, NF, FI, PRE, 2.0f, 1.0f, 1024, 0.222f, 32, 64, 4, 32},
    {0, NF, FI, AT, 2.0f, 1.0f, 512, 0.222f, 128, 64, 4, 32},
    {2, NF, FI, PRE, 0.5f, 1.0f, 256, 0.5f, 32, 64, 4, 32},
    {0, NF, FI, AT, 0.5f, 1.0f, 256, 0.5f, 32, 64, 4, 32},
    {1, NF, FI, PRE, 1.0f, 1.0f, 512, 0.75f, 32, 64, 4, 32},
    {0, NF, FI, AT, 8.0f, 1.0f, 2048, 0.222f, 32, 64, 4, 32},
    {1, NF, FI, AT, 0.5f, 1.0f, 128, 0.5f, 32, 64, 4, 32},
    {0, NF, FI, AT, 2.0f, 1.0f, 1024, 0.5f, 32, 64, 4, 32},
    // near-far over the bucket queue
    {1, NF, DQ, PRE, 0.5f, 0.5f, 128, 0.5f, 32, 64, 4, 32},
    {1, NF, DQ, PRE, 0.5f, 2.0f, 256, 0.5f, 64, 64, 4, 32},
    {0, NF, DQ, AT, 2.0f, 4.0f, 1024, 0.222f, 32, 64, 2, 32},
    {0, NF, DQ, AT, 1.0f, 2.0f, 1024, 0.333f, 32, 64, 4, 32},
    {0, NF, DQ, AT, 2.0f, 8.0f, 1024, 0.222f, 32, 64, 8, 32},
    {1, NF, DQ, PRE, 1.0f, 1.0f, 256, 0.25f, 32, 64, 2, 32},
    {0, NF, DQ, PRE, 2.0f, 4.0f, 512, 0.5f, 32, 64, 4, 32},
    {0, NF, DQ, AT, 0.5f, 1.0f, 256, 0.222f, 32, 64, 4, 32},
    // filter queue
    {1, FQ, FI, PRE, 0.5f, 1.0f, 256, 0.5f, 32, 64, 4, 32},
    {0, FQ, FI, AT, 2.0f, 1.0f, 1024, 0.222f, 32, 64, 4, 32},
    {0, FQ, DQ, AT, 1.0f, 2.0f, 1024, 0.222f, 32, 64, 4, 32},
    {1, FQ, DQ, PRE, 0.5f, 1.0f, 256, 0.5f, 32, 64, 4, 32},
    {0, FQ, FI, AT, 4.0f, 1.0f, 1024, 0.333f, 32, 64, 4, 32},
    {1, FQ, DQ, PRE, 2.0f, 4.0f, 512, 0.25f, 32, 64, 2, 32},
    // small-label-first deque
    {1, SLF, FI, PRE, 1.0f, 1.0f, 128, 0.5f, 32, 64, 4, 32},
    {1, SLF, FI, PRE, 1.0f, 1.0f, 256, 0.5f, 64, 64, 4, 32},
    {2, SLF, FI, PRE, 1.0f, 1.0f, 256, 0.5f, 32, 64, 4, 32},
    {0, SLF, FI, AT, 1.0f, 1.0f, 1024, 0.222f, 32, 64, 4, 32},
    {1, SLF, DQ, PRE, 1.0f, 1.0f, 256, 0.5f, 32, 64, 4, 32},
    {0, SLF, DQ, AT, 1.0f, 4.0f, 1024, 0.222f, 32, 64, 4, 32},
    // FIFO vector with periodic flush
    {1, V, FI, PRE, 1.0f, 1.0f, 256, 0.5f, 32, 8, 4, 32},
    {1, V, FI, PRE, 1.0f, 1.0f, 256, 0.5f, 32, 64, 4, 32},
    {0, V, FI, AT, 1.0f, 1.0f, 1024, 0.222f, 32, 32, 4, 32},
    {2, V, FI, PRE, 1.0f, 1.0f, 512, 0.5f, 32, 32, 4, 32},
    {1, V, DQ, PRE, 1.0f, 1.0f, 256, 0.5f, 32, 64, 4, 32},
    {0, V, DQ, AT, 1.0f, 4.0f, 1024, 0.222f, 32, 32, 4, 32},
    // spill-threshold and whole-wave-threshold variants
    {1, NF, FI, PRE, 0.5f, 1.0f, 256, 0.5f, 128, 64, 4, 32},
    {0, NF, FI, AT, 2.0f, 1.0f, 1024, 0.222f, 128, 64, 4, 32},
    {1, NF, FI, PRE, 0.5f, 1.0f, 256, 0.5f, 64, 64, 4, 256},
    {1, NF, FI, PRE, 0.5f, 1.0f, 128, 0.333f, 32, 64, 4, 128},
    // register queues only, and one global FIFO alone
    {2, N, FI, PRE, 1.0f, 1.0f, 64, 0.5f, 32, 64, 4, 32},
    {0, N, FI, AT, 1.0f, 1.0f, 64, 0.222f, 32, 64, 4, 32},
};
constexpr int kNumTemplates = (int)(sizeof(kTemplates) / sizeof(kTemplates[0]));

// Trained forest (generated by the selector's training script from timings
// of every template on a seeded synthetic corpus).
#include "mlmq_selector_model.inc"

static_assert(kSelInputs == 20, "model inputs");

float safe_log2(double x) { return (float)std::log2(std::max(x, 1e-9)); }

// Model inputs for template t on a graph with features f: the Table 2
// features (sizes as log2, degree and weight spread relative to their means)
// then the template's knobs.
void sel_inputs(const mlmq_features& f, const Template& t, float* x) {
  x[0] = safe_log2(std::max(1.0, f.n));
  x[1] = safe_log2(std::max(1.0, f.nnz));
  x[2] = (float)f.avg_deg;
  x[3] = safe_log2(std::max(1.0, f.max_deg));
  x[4] = (float)(f.std_deg / std::max(f.avg_deg, 1e-9));
  x[5] = safe_log2(std::max(1.0, f.avg_w));
  x[6] = (float)(f.std_w / std::max(f.avg_w, 1e-9));
  x[7] = safe_log2(std::max(1.0, f.max_w));
  x[8] = (float)t.l0;
  x[9] = (float)t.l1;
  x[10] = (float)t.l2;
  x[11] = (float)t.relax;
  x[12] = safe_log2(t.d1m);
  x[13] = safe_log2(t.d2m);
  x[14] = safe_log2(t.cap);
  x[15] = t.grid;
  x[16] = safe_log2(t.donate);
  x[17] = safe_log2(t.wb);
  x[18] = (float)t.bnum;
  x[19] = safe_log2(t.thv);
}

// Mean of the trees' leaf values. Inputs are compared as float against
// double thresholds, as the training library does.
double sel_predict(const float* x) {
  if (kSelTrees == 0) return 0.0;
  double s = 0;
  for (int tr = 0; tr < kSelTrees; ++tr) {
    int32_t i = kSelRoot[tr];
    while (kSelFeat[i] >= 0) i = kSelRoot[tr] + ((double)x[kSelFeat[i]] <= kSelThr[i] ? kSelLeft[i] : kSelRight[i]);
    s += kSelValue[i];
  }
  return s / kSelTrees;
}

// Template ids ordered by predicted relative performance (best first; ties
// keep list order).
std::vector<int32_t> ranked(const mlmq_features& f, std::vector<float>* scores) {
  std::vector<float> sc((size_t)kNumTemplates);
  float x[kSelInputs];
  for (int t = 0; t < kNumTemplates; ++t) {
    sel_inputs(f, kTemplates[t], x);
    sc[t] = (float)sel_predict(x);
  }
  std::vector<int32_t> order((size_t)kNumTemplates);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return sc[a] > sc[b]; });
  if (scores) *scores = sc;
  return order;
}

uint32_t pow2_log_nearest(double x) {
  const double l = std::log2(std::max(x, 1.0));
  return (uint32_t)std::min(31.0, std::max(0.0, std::floor(l + 0.5)));
}

}  // namespace

namespace mlmq {

int32_t selector_pick(const mlmq_features& f) { return kSelTrees ? ranked(f, nullptr)[0] : -1; }

// Template t (or the feature-driven default for t = -1) as a config for g.
int template_config(const mlmq_graph* g, int32_t t, mlmq_config* out) {
  mlmq_config c;
  c.struct_size = sizeof(mlmq_config);
  default_config(&c);
  heuristic_config(g, &c);
  if (t >= 0) {
    const Template& p = kTemplates[t];
    const double mw = std::max(1.0, g->features.avg_w);
    c.l0_rows = p.l0;
    c.l1_type = p.l1;
    c.l2_type = p.l2;
    c.relax_mode = p.relax;
    c.delta1 = (uint32_t)std::max(1.0, std::floor(mw * p.d1m + 0.5));
    c.delta2_log2 = pow2_log_nearest(mw * p.d2m);
    c.l1_cap = p.cap;
    c.l1_flush_wb = p.wb;
    c.bmax = 32;
    c.bnum = p.bnum;
    c.th_v = p.thv;
    c.donate_min = p.donate;
    const uint32_t slots = 12u * (uint32_t)std::max(1, device_info()->cus);
    c.grid_wgs = std::max<uint32_t>(64, (uint32_t)std::floor(p.grid * slots + 0.5f));
  }
  const int rc = check_config(&c);
  if (rc) return rc;
  *out = c;
  return MLMQ_OK;
}

}  // namespace mlmq

namespace {

void keep_caller_fields(mlmq_config* out, const mlmq_config& c) {
  mlmq_stats* so = out->stats_out;
  void* ss = out->stream;
  *out = c;
  out->stats_out = so;
  out->stream = ss;
}

}  // namespace

extern "C" int32_t mlmq_candidate_count(void) { return kNumTemplates; }

extern "C" int mlmq_select_inputs(const mlmq_features* f, int32_t t, float* x) {
  if (!f || !x) return set_error(MLMQ_ERR_INVALID_ARG, "NULL argument");
  if (t < 0 || t >= kNumTemplates) return set_error(MLMQ_ERR_INVALID_ARG, "template %d out of range", t);
  sel_inputs(*f, kTemplates[t], x);
  return MLMQ_OK;
}

extern "C" int mlmq_select_rank(const mlmq_features* f, int32_t* order, float* scores, int32_t cap) {
  if (!f || cap < 0 || (cap > 0 && !order)) return set_error(MLMQ_ERR_INVALID_ARG, "NULL argument");
  std::vector<float> sc;
  const std::vector<int32_t> ord = ranked(*f, &sc);
  for (int32_t i = 0; i < cap && i < kNumTemplates; ++i) order[i] = ord[i];
  if (scores)
    for (int t = 0; t < kNumTemplates; ++t) scores[t] = sc[t];
  return MLMQ_OK;
}

extern "C" int mlmq_candidate_config(const mlmq_graph* g, int32_t t, mlmq_config* out) {
  if (!g || !out) return set_error(MLMQ_ERR_INVALID_ARG, "NULL argument");
  if (out->struct_size != sizeof(mlmq_config))
    return set_error(MLMQ_ERR_INVALID_ARG, "config struct_size %u != %zu", out->struct_size, sizeof(mlmq_config));
  if (t < -1 || t >= kNumTemplates) return set_error(MLMQ_ERR_INVALID_ARG, "template %d out of range", t);
  int rc = need_device();
  if (rc) return rc;
  mlmq_config c;
  rc = template_config(g, t, &c);
  if (rc) return rc;
  keep_caller_fields(out, c);
  return MLMQ_OK;
}

extern "C" int mlmq_select(const mlmq_graph* g, mlmq_config* out) {
  if (!g || !out) return set_error(MLMQ_ERR_INVALID_ARG, "NULL argument");
  if (out->struct_size != sizeof(mlmq_config))
    return set_error(MLMQ_ERR_INVALID_ARG, "config struct_size %u != %zu", out->struct_size, sizeof(mlmq_config));
  int rc = need_device();
  if (rc) return rc;
  const int32_t t = selector_pick(g->features);
  mlmq_config c;
  rc = template_config(g, t, &c);
  if (rc) return rc;
  keep_caller_fields(out, c);
  return MLMQ_OK;
}

// ------------------------------------------------------------ autotuner

extern "C" int mlmq_autotune(mlmq_graph* g, uint32_t budget_ms, mlmq_config* out) {
  if (!g) return set_error(MLMQ_ERR_INVALID_ARG, "graph is NULL");
  if (out && out->struct_size != sizeof(mlmq_config))
    return set_error(MLMQ_ERR_INVALID_ARG, "config struct_size %u != %zu", out->struct_size, sizeof(mlmq_config));
  int rc = need_device();
  if (rc) return rc;
  if (!budget_ms) budget_ms = 2000;
  uint32_t* d_dist = nullptr;
  hipError_t e = hipMalloc(&d_dist, 4ull * g->n);
  if (e != hipSuccess) return hip_fail(e, "autotune buffer");
  // Seeded sources: the highest-degree vertex plus two spread by a fixed LCG
  // among vertices with out-degree >= 1 (located on the host copy of offsets).
  std::vector<int32_t> off((size_t)g->n + 1);
  e = hipMemcpy(off.data(), g->d_off, 4ull * (g->n + 1), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    (void)hipFree(d_dist);
    return hip_fail(e, "autotune offsets");
  }
  std::vector<uint32_t> srcs;
  int32_t best_v = 0, best_d = -1;
  for (int32_t u = 0; u < g->n; ++u)
    if (off[u + 1] - off[u] > best_d) {
      best_d = off[u + 1] - off[u];
      best_v = u;
    }
  srcs.push_back((uint32_t)best_v);
  uint64_t x = 0x2545F4914F6CDD1Dull;
  for (int tries = 0; srcs.size() < 3 && tries < 1000; ++tries) {
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    const uint32_t u = (uint32_t)((x >> 33) % (uint64_t)g->n);
    if (off[u + 1] > off[u]) srcs.push_back(u);
  }
  // Candidates: the feature-driven default, then the templates in the
  // selector's order (with no trained model, in list order). Each is timed on
  // the sources until the budget is spent.
  std::vector<int32_t> cand = {-1};
  for (int32_t t : ranked(g->features, nullptr)) cand.push_back(t);
  const auto t0 = std::chrono::steady_clock::now();
  double best_ms = 1e300;
  mlmq_config best;
  rc = template_config(g, -1, &best);
  if (rc) {
    (void)hipFree(d_dist);
    return rc;
  }
  for (size_t ci = 0; ci < cand.size(); ++ci) {
    const double el = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (ci > 0 && el > budget_ms) break;
    mlmq_config c;
    if (template_config(g, cand[ci], &c) != MLMQ_OK) continue;
    const mlmq_config keep = c;
    mlmq_stats st;
    std::memset(&st, 0, sizeof(st));
    st.struct_size = sizeof(st);
    c.stats_out = &st;
    c.stream = out ? out->stream : nullptr;
    // a poor candidate may not take more than the whole budget, nor much
    // longer than the best so far
    uint32_t lim = std::max<uint32_t>(200, budget_ms);
    if (best_ms < 1e299) lim = std::min<uint32_t>(lim, (uint32_t)(4.0 * best_ms) + 50);
    c.timeout_ms = std::min<uint32_t>(c.timeout_ms ? c.timeout_ms : 60000, lim);
    c.max_retries = 1;
    double total = 0;
    bool okc = true;
    for (uint32_t s : srcs) {
      if (run_single(g, s, d_dist, c) != MLMQ_OK) {
        okc = false;
        break;
      }
      total += st.kernel_ms;
    }
    if (okc && total < best_ms) {
      best_ms = total;
      best = keep;
    }
  }
  (void)hipFree(d_dist);
  best.stats_out = nullptr;
  best.stream = nullptr;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    g->tuned = best;
    g->has_tuned = true;
  }
  if (out) keep_caller_fields(out, best);
  return MLMQ_OK;
}
