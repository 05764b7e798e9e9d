"""Failed conditions of the optimality check (mlmq_check), counted directly
with numpy: edges (u, v, w) with dist[u] finite whose dist[v] is infinite or
above dist[u] + w, vertices other than the source with a finite distance and
no tight in-edge, and 1 if dist[source] != 0."""
import numpy as np


def check_count(csr, src, d):
    d64 = np.asarray(d).astype(np.int64)
    inf = np.int64(0xFFFFFFFF)
    u = np.repeat(np.arange(csr.n), np.diff(csr.off))
    v = np.asarray(csr.col, np.int64)
    s = d64[u] + np.asarray(csr.w, np.int64)
    fin = d64[u] != inf
    bad_edges = int(np.count_nonzero(fin & ((d64[v] == inf) | (d64[v] > s))))
    tight = np.zeros(csr.n, bool)
    tight[v[fin & (d64[v] == s)]] = True
    others = np.arange(csr.n) != src
    bad_vertices = int(np.count_nonzero(others & (d64 != inf) & ~tight))
    return bad_edges + bad_vertices + int(d64[src] != 0)
