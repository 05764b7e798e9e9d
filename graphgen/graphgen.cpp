// Seeded synthetic graph generator (CSR, host only).
//
// Input generation only: this file holds none of the shortest-path arithmetic.
// Both the CPU oracle and the GPU path are fed from what it writes.
//
// Every random draw is a counter-based hash of (seed, stream, index), so a graph
// is a pure function of its parameters: bit-reproducible, independent of thread
// count and of the order in which edges are produced.
//
// Graph shapes (stand-ins for the paper's workloads, Section 5.1 / Table 4):
//   * 2-D grid with 4-neighbour edges, optional independent drop of each
//     undirected edge (road-like when p_drop > 0, mesh-like when 0).
//   * RMAT (a,b,c,d) tuples, symmetrised, self-loops and duplicates removed,
//     vertex ids scrambled by a seeded bijection (Graph500-style permutation).
//   * uniform random directed pairs, self-loops and duplicates removed.
// Weights: 1 + (hash mod wmax) per undirected pair keyed by (min(u,v), max(u,v)),
// so both directions of an edge carry the same weight.
//
// Output CSR: row_offsets int64[n+1], col int32[m], w uint32[m]; every row sorted
// by destination id.

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t kStreamDrop = 0x64726f70ULL;     // "drop"
constexpr uint64_t kStreamWeight = 0x77656967ULL;   // "weig"
constexpr uint64_t kStreamRmat = 0x726d6174ULL;     // "rmat"
constexpr uint64_t kStreamPerm = 0x7065726dULL;     // "perm"
constexpr uint64_t kStreamUni = 0x756e6966ULL;      // "unif"

inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

// One 64-bit draw for (seed, stream, index).
inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t index) {
  return splitmix64(splitmix64(seed ^ splitmix64(stream)) + index);
}

inline uint32_t pair_weight(uint64_t seed, uint32_t u, uint32_t v, uint32_t wmax) {
  uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
  uint64_t h = draw(seed, kStreamWeight, (hi << 32) | lo);
  return 1u + (uint32_t)(h % (uint64_t)wmax);
}

// Bijection on [0, 2^bits): alternating xorshift and odd multiplication, both
// invertible modulo 2^bits.
struct Scrambler {
  uint32_t bits;
  uint64_t mask, mul[3], add[3];
  Scrambler(uint64_t seed, uint32_t b) : bits(b) {
    mask = b >= 64 ? ~0ULL : ((1ULL << b) - 1);
    for (int r = 0; r < 3; ++r) {
      mul[r] = draw(seed, kStreamPerm, 2 * r) | 1ULL;
      add[r] = draw(seed, kStreamPerm, 2 * r + 1);
    }
  }
  uint64_t operator()(uint64_t x) const {
    if (bits == 0) return 0;
    uint32_t sh = bits / 2 ? bits / 2 : 1;
    for (int r = 0; r < 3; ++r) {
      x = (x * mul[r]) & mask;
      x = (x + add[r]) & mask;
      x ^= x >> sh;
    }
    return x;
  }
};

// Build a CSR from a directed pair list: optional symmetrisation, self-loop
// removal, de-duplication, per-row sort, weight assignment.
struct PairCsr {
  int64_t n = 0, m = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> col;
  std::vector<uint32_t> w;
};

void build_csr(int64_t n, const uint32_t* src, const uint32_t* dst, int64_t npairs, bool symmetrize,
               uint64_t seed, uint32_t wmax, PairCsr* out) {
  std::vector<std::atomic<uint32_t>> deg(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) deg[i].store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npairs; ++i) {
    uint32_t u = src[i], v = dst[i];
    if (u == v) continue;
    deg[u].fetch_add(1, std::memory_order_relaxed);
    if (symmetrize) deg[v].fetch_add(1, std::memory_order_relaxed);
  }
  std::vector<int64_t> tmp_off(n + 1);
  tmp_off[0] = 0;
  for (int64_t i = 0; i < n; ++i) tmp_off[i + 1] = tmp_off[i] + deg[i].load(std::memory_order_relaxed);
  std::vector<uint32_t> tmp(tmp_off[n]);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) deg[i].store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npairs; ++i) {
    uint32_t u = src[i], v = dst[i];
    if (u == v) continue;
    tmp[tmp_off[u] + deg[u].fetch_add(1, std::memory_order_relaxed)] = v;
    if (symmetrize) tmp[tmp_off[v] + deg[v].fetch_add(1, std::memory_order_relaxed)] = u;
  }
  std::vector<int64_t> ndeg(n);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    uint32_t* b = tmp.data() + tmp_off[i];
    uint32_t* e = tmp.data() + tmp_off[i + 1];
    std::sort(b, e);
    ndeg[i] = std::unique(b, e) - b;
  }
  out->n = n;
  out->off.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) out->off[i + 1] = out->off[i] + ndeg[i];
  out->m = out->off[n];
  out->col.resize(out->m);
  out->w.resize(out->m);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t* b = tmp.data() + tmp_off[i];
    int64_t o = out->off[i];
    for (int64_t k = 0; k < ndeg[i]; ++k) {
      out->col[o + k] = (int32_t)b[k];
      out->w[o + k] = pair_weight(seed, (uint32_t)i, b[k], wmax);
    }
  }
}

thread_local PairCsr g_last;

void hand_out(int64_t* n, int64_t* m) {
  *n = g_last.n;
  *m = g_last.m;
}

}  // namespace

extern "C" {

// Library version of the draw, exposed so tests can check reproducibility.
uint64_t gg_draw(uint64_t seed, uint64_t stream, uint64_t index) { return draw(seed, stream, index); }

int gg_set_threads(int t) {
  if (t > 0) omp_set_num_threads(t);
  return omp_get_max_threads();
}

// R x C grid, vertex id r*C + c. Each undirected edge is dropped independently
// with probability p_drop. Returns the number of directed edges, or -1.
int64_t gg_grid(int64_t rows, int64_t cols, double p_drop, uint32_t wmax, uint64_t seed,
                int64_t* off, int32_t* col, uint32_t* w) {
  if (rows <= 0 || cols <= 0 || wmax == 0) return -1;
  const int64_t n = rows * cols;
  const uint64_t thr = p_drop <= 0.0 ? 0 : (p_drop >= 1.0 ? ~0ULL : (uint64_t)(p_drop * 18446744073709551616.0));
  auto kept = [&](int64_t a, int64_t b) -> bool {
    if (thr == 0) return true;
    if (thr == ~0ULL) return false;
    uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    return draw(seed, kStreamDrop, (hi << 32) | lo) >= thr;
  };
  // neighbours in increasing id order: up, left, right, down
  auto for_nbrs = [&](int64_t u, auto&& f) {
    int64_t r = u / cols, c = u % cols;
    if (r > 0 && kept(u, u - cols)) f(u - cols);
    if (c > 0 && kept(u, u - 1)) f(u - 1);
    if (c + 1 < cols && kept(u, u + 1)) f(u + 1);
    if (r + 1 < rows && kept(u, u + cols)) f(u + cols);
  };
  std::vector<int64_t> deg(n);
#pragma omp parallel for schedule(static)
  for (int64_t u = 0; u < n; ++u) {
    int64_t d = 0;
    for_nbrs(u, [&](int64_t) { ++d; });
    deg[u] = d;
  }
  int64_t total = 0;
  for (int64_t u = 0; u < n; ++u) {
    if (off) off[u] = total;
    total += deg[u];
  }
  if (off) off[n] = total;
  if (!col || !w) return total;
#pragma omp parallel for schedule(static)
  for (int64_t u = 0; u < n; ++u) {
    int64_t o = off[u];
    for_nbrs(u, [&](int64_t v) {
      col[o] = (int32_t)v;
      w[o] = pair_weight(seed, (uint32_t)u, (uint32_t)v, wmax);
      ++o;
    });
  }
  return total;
}

// RMAT: ef * 2^scale tuples, each bit level picks a quadrant with
// probabilities (a, b, c, 1-a-b-c). Symmetrised, self-loops/duplicates
// removed, ids scrambled when permute != 0. The result is held per thread
// until gg_take is called. Returns 0 or -1.
int gg_rmat_build(int scale, int64_t edge_factor, double a, double b, double c, int permute,
                  uint32_t wmax, uint64_t seed, int64_t* n_out, int64_t* m_out) {
  if (scale < 1 || scale > 30 || edge_factor < 1 || wmax == 0) return -1;
  const int64_t n = 1LL << scale;
  const int64_t M = edge_factor * n;
  const double ab = a + b, abc = a + b + c;
  std::vector<uint32_t> src(M), dst(M);
  Scrambler scr(seed, scale);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < M; ++i) {
    uint64_t u = 0, v = 0;
    for (int l = 0; l < scale; ++l) {
      double r = (double)(draw(seed, kStreamRmat, (uint64_t)i * 64 + l) >> 11) * (1.0 / 9007199254740992.0);
      uint64_t bu = r >= ab ? 1 : 0;
      uint64_t bv = (r >= a && r < ab) || r >= abc ? 1 : 0;
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    if (permute) {
      u = scr(u);
      v = scr(v);
    }
    src[i] = (uint32_t)u;
    dst[i] = (uint32_t)v;
  }
  build_csr(n, src.data(), dst.data(), M, true, seed, wmax, &g_last);
  hand_out(n_out, m_out);
  return 0;
}

// Uniform random directed pairs: npairs (u, v) drawn uniformly from [0, n)^2,
// self-loops/duplicates removed (not symmetrised). Returns 0 or -1.
int gg_uniform_build(int64_t n, int64_t npairs, uint32_t wmax, uint64_t seed, int64_t* n_out,
                     int64_t* m_out) {
  if (n < 1 || n > (1LL << 31) || npairs < 0 || wmax == 0) return -1;
  std::vector<uint32_t> src(npairs), dst(npairs);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npairs; ++i) {
    src[i] = (uint32_t)(draw(seed, kStreamUni, 2 * (uint64_t)i) % (uint64_t)n);
    dst[i] = (uint32_t)(draw(seed, kStreamUni, 2 * (uint64_t)i + 1) % (uint64_t)n);
  }
  build_csr(n, src.data(), dst.data(), npairs, false, seed, wmax, &g_last);
  hand_out(n_out, m_out);
  return 0;
}

// Copy the graph held by gg_*_build into caller buffers (off[n+1], col[m],
// w[m]) and release it.
int gg_take(int64_t* off, int32_t* col, uint32_t* w) {
  const int64_t n = g_last.n, m = g_last.m;
  std::memcpy(off, g_last.off.data(), sizeof(int64_t) * (n + 1));
  std::memcpy(col, g_last.col.data(), sizeof(int32_t) * m);
  std::memcpy(w, g_last.w.data(), sizeof(uint32_t) * m);
  g_last = PairCsr();
  return 0;
}

}  // extern "C"
