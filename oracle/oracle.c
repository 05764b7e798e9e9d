/*
 * CPU oracle for single-source shortest paths (SSSP).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library. The GPU library
 * never calls it and shares no code, header, table or helper with it.
 *
 * What it computes (Section 2.1, problem statement): for a directed graph
 * G(V, E, W) with non-negative integer weights and a source s, the vector
 * L(s) of shortest path lengths l_su for every u in V, i.e.
 *     dist[u] = min over all s->u paths of the sum of edge weights,
 * and UINT32_MAX (0xFFFFFFFF) where no path exists. The minimum is unique, so
 * any correct schedule of relaxations (Dijkstra, Bellman-Ford, MLMQ) must give
 * this exact vector.
 *
 * Reading of the paper (it gives `int dist` in its kernel sketch and no
 * sentinel): distances are uint32, UINT32_MAX marks "unreachable", the largest
 * representable finite distance is 2^32 - 2. Arithmetic here is uint64, so
 * sums never wrap; a finite true distance >= 2^32 - 1 is reported as overflow.
 *
 * Functions:
 *   oracle_dijkstra      textbook Dijkstra (Section 2.1: priority queue, the
 *                        work-optimal endpoint) with a binary min-heap and lazy
 *                        deletion of stale entries.
 *   oracle_bellman_ford  textbook Bellman-Ford (Section 2.1: the maximally
 *                        parallel endpoint): repeat a full pass relaxing every
 *                        edge until nothing changes. Used as an independent
 *                        brute-force check on small graphs.
 *   oracle_certificate   optimality certificate: a vector passes iff it equals
 *                        the shortest-distance vector (proof in the comment).
 *   oracle_reach_stats   n_reach / m_reach of a distance vector (edges counted
 *                        once per directed edge out of a reachable vertex).
 *   oracle_bfs           breadth-first search levels (Section 5.7's BFS case
 *                        study): the fewest edges on a path from s, by the
 *                        textbook FIFO-queue traversal.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_ERR_INVALID_ARG (-1)
#define ORACLE_ERR_OUT_OF_MEMORY (-2)
#define ORACLE_ERR_DISTANCE_OVERFLOW (-3)
#define ORACLE_CERT_BAD_SOURCE (-10)
#define ORACLE_CERT_EDGE_VIOLATED (-11)
#define ORACLE_CERT_UNSUPPORTED (-12)

#define INF32 0xFFFFFFFFu
#define INF64 0xFFFFFFFFFFFFFFFFull

static int check_csr(int64_t n, const int64_t* off, const int32_t* col, int64_t src) {
  if (n < 1 || !off || src < 0 || src >= n) return ORACLE_ERR_INVALID_ARG;
  if (off[0] != 0) return ORACLE_ERR_INVALID_ARG;
  for (int64_t u = 0; u < n; ++u)
    if (off[u + 1] < off[u]) return ORACLE_ERR_INVALID_ARG;
  for (int64_t e = 0; e < off[n]; ++e)
    if (col[e] < 0 || col[e] >= n) return ORACLE_ERR_INVALID_ARG;
  return ORACLE_OK;
}

/* Write a uint64 distance vector out as uint32 with UINT32_MAX = unreachable. */
static int narrow(int64_t n, const uint64_t* d64, uint32_t* dist_out) {
  int rc = ORACLE_OK;
  for (int64_t u = 0; u < n; ++u) {
    if (d64[u] == INF64) {
      dist_out[u] = INF32;
    } else if (d64[u] >= (uint64_t)INF32) {
      dist_out[u] = INF32;
      rc = ORACLE_ERR_DISTANCE_OVERFLOW;
    } else {
      dist_out[u] = (uint32_t)d64[u];
    }
  }
  return rc;
}

/* ---- Dijkstra with a binary min-heap keyed on tentative distance ---- */

typedef struct {
  uint64_t d;
  int64_t v;
} heap_item;

typedef struct {
  heap_item* a;
  int64_t size, cap;
} heap;

static int heap_push(heap* h, uint64_t d, int64_t v) {
  if (h->size == h->cap) {
    int64_t nc = h->cap ? 2 * h->cap : 1024;
    heap_item* na = (heap_item*)realloc(h->a, (size_t)nc * sizeof(heap_item));
    if (!na) return ORACLE_ERR_OUT_OF_MEMORY;
    h->a = na;
    h->cap = nc;
  }
  int64_t i = h->size++;
  while (i > 0) { /* sift up */
    int64_t p = (i - 1) / 2;
    if (h->a[p].d <= d) break;
    h->a[i] = h->a[p];
    i = p;
  }
  h->a[i].d = d;
  h->a[i].v = v;
  return ORACLE_OK;
}

static heap_item heap_pop(heap* h) {
  heap_item top = h->a[0];
  heap_item last = h->a[--h->size];
  int64_t i = 0;
  for (;;) { /* sift down */
    int64_t l = 2 * i + 1, r = l + 1, s = i;
    uint64_t ds = last.d;
    if (l < h->size && h->a[l].d < ds) { s = l; ds = h->a[l].d; }
    if (r < h->size && h->a[r].d < ds) { s = r; }
    if (s == i) break;
    h->a[i] = h->a[s];
    i = s;
  }
  if (h->size > 0) h->a[i] = last;
  return top;
}

/*
 * Dijkstra: repeatedly settle the queued vertex of smallest tentative distance
 * and relax its out-edges (if d(u) + w < d(v), lower d(v) and queue v). A popped
 * pair whose distance is larger than the vertex's current label is stale and
 * skipped (lazy deletion instead of decrease-key).
 */
int oracle_dijkstra(int64_t n, const int64_t* off, const int32_t* col, const uint32_t* w, int64_t src,
                    uint32_t* dist_out) {
  int rc = check_csr(n, off, col, src);
  if (rc) return rc;
  uint64_t* d = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
  if (!d) return ORACLE_ERR_OUT_OF_MEMORY;
  for (int64_t u = 0; u < n; ++u) d[u] = INF64;
  heap h = {0, 0, 0};
  d[src] = 0;
  rc = heap_push(&h, 0, src);
  while (rc == ORACLE_OK && h.size > 0) {
    heap_item it = heap_pop(&h);
    if (it.d > d[it.v]) continue; /* stale entry */
    for (int64_t e = off[it.v]; e < off[it.v + 1]; ++e) {
      int64_t v = col[e];
      uint64_t nd = it.d + (uint64_t)w[e];
      if (nd < d[v]) {
        d[v] = nd;
        rc = heap_push(&h, nd, v);
        if (rc) break;
      }
    }
  }
  free(h.a);
  if (rc == ORACLE_OK) rc = narrow(n, d, dist_out);
  free(d);
  return rc;
}

/*
 * Bellman-Ford: start from d(s) = 0, everything else infinite; sweep all edges
 * relaxing each one, and repeat until a sweep changes nothing. With
 * non-negative weights this ends after at most n sweeps.
 */
int oracle_bellman_ford(int64_t n, const int64_t* off, const int32_t* col, const uint32_t* w, int64_t src,
                        uint32_t* dist_out) {
  int rc = check_csr(n, off, col, src);
  if (rc) return rc;
  uint64_t* d = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
  if (!d) return ORACLE_ERR_OUT_OF_MEMORY;
  for (int64_t u = 0; u < n; ++u) d[u] = INF64;
  d[src] = 0;
  for (int64_t pass = 0; pass <= n; ++pass) {
    int changed = 0;
    for (int64_t u = 0; u < n; ++u) {
      if (d[u] == INF64) continue;
      for (int64_t e = off[u]; e < off[u + 1]; ++e) {
        uint64_t nd = d[u] + (uint64_t)w[e];
        if (nd < d[col[e]]) {
          d[col[e]] = nd;
          changed = 1;
        }
      }
    }
    if (!changed) break;
  }
  rc = narrow(n, d, dist_out);
  free(d);
  return rc;
}

/*
 * Optimality certificate for a claimed distance vector D (uint32, UINT32_MAX
 * = unreachable). D passes iff
 *   (1) D[s] = 0;
 *   (2) for every edge (u, v, w) with D[u] finite: D[v] is finite and
 *       D[v] <= D[u] + w (evaluated in uint64);
 *   (3) every vertex with finite D is reached from s by a BFS that follows only
 *       tight edges (D[u] finite and D[u] + w == D[v]).
 * Why this is exactly the shortest-distance vector d: by (3) each finite D[v]
 * is the length of a real s->v path, so D[v] >= d(v) and every finite vertex
 * is reachable. By (1)-(2) and induction along a shortest path, every
 * reachable v has D[v] finite and D[v] <= d(v). Hence D[v] = d(v) on the
 * reachable set and D[v] = UINT32_MAX elsewhere. The BFS (rather than "has a
 * tight in-edge") rules out zero-weight cycles that support themselves.
 * Clause (2) also catches overflow: a reachable vertex whose true distance is
 * >= 2^32 - 1 can only be reported as UINT32_MAX, which (2) rejects.
 * On failure *where receives the offending vertex. *depth receives the largest
 * BFS level (fewest-hop depth of the shortest-path DAG) when it passes.
 */
int oracle_certificate(int64_t n, const int64_t* off, const int32_t* col, const uint32_t* w, int64_t src,
                       const uint32_t* D, int64_t* where, int64_t* depth) {
  int rc = check_csr(n, off, col, src);
  if (rc) return rc;
  if (where) *where = -1;
  if (depth) *depth = 0;
  if (D[src] != 0) {
    if (where) *where = src;
    return ORACLE_CERT_BAD_SOURCE;
  }
  for (int64_t u = 0; u < n; ++u) {
    if (D[u] == INF32) continue;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      uint32_t dv = D[col[e]];
      if (dv == INF32 || (uint64_t)dv > (uint64_t)D[u] + (uint64_t)w[e]) {
        if (where) *where = col[e];
        return ORACLE_CERT_EDGE_VIOLATED;
      }
    }
  }
  int64_t* q = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* level = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!q || !level) {
    free(q);
    free(level);
    return ORACLE_ERR_OUT_OF_MEMORY;
  }
  for (int64_t u = 0; u < n; ++u) level[u] = -1;
  int64_t qh = 0, qt = 0;
  q[qt++] = src;
  level[src] = 0;
  int32_t maxlev = 0;
  while (qh < qt) {
    int64_t u = q[qh++];
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      int64_t v = col[e];
      if (level[v] < 0 && (uint64_t)D[u] + (uint64_t)w[e] == (uint64_t)D[v]) {
        level[v] = level[u] + 1;
        if (level[v] > maxlev) maxlev = level[v];
        q[qt++] = v;
      }
    }
  }
  rc = ORACLE_OK;
  for (int64_t u = 0; u < n; ++u) {
    if (D[u] != INF32 && level[u] < 0) {
      if (where) *where = u;
      rc = ORACLE_CERT_UNSUPPORTED;
      break;
    }
  }
  if (rc == ORACLE_OK && depth) *depth = maxlev;
  free(q);
  free(level);
  return rc;
}

/* Number of vertices with finite distance, and directed edges leaving them. */
int oracle_reach_stats(int64_t n, const int64_t* off, const uint32_t* D, int64_t* n_reach, int64_t* m_reach) {
  if (n < 1 || !off || !D) return ORACLE_ERR_INVALID_ARG;
  int64_t nr = 0, mr = 0;
  for (int64_t u = 0; u < n; ++u) {
    if (D[u] != INF32) {
      ++nr;
      mr += off[u + 1] - off[u];
    }
  }
  if (n_reach) *n_reach = nr;
  if (m_reach) *m_reach = mr;
  return ORACLE_OK;
}

/* Breadth-first search: level[s] = 0; a vertex first reached from a vertex of
 * level k gets level k + 1; vertices never reached keep UINT32_MAX. The FIFO
 * queue visits vertices in non-decreasing level order, so the first time a
 * vertex is reached is along a fewest-edge path. */
int oracle_bfs(int64_t n, const int64_t* off, const int32_t* col, int64_t src, uint32_t* level) {
  int rc = check_csr(n, off, col, src);
  if (rc != ORACLE_OK) return rc;
  if (!level) return ORACLE_ERR_INVALID_ARG;
  int64_t* queue = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!queue) return ORACLE_ERR_OUT_OF_MEMORY;
  for (int64_t v = 0; v < n; ++v) level[v] = INF32;
  int64_t head = 0, tail = 0;
  level[src] = 0;
  queue[tail++] = src;
  while (head < tail) {
    const int64_t u = queue[head++];
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      const int64_t v = col[e];
      if (level[v] == INF32) {
        level[v] = level[u] + 1;
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return ORACLE_OK;
}
