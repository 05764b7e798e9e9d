"""Pins for the CPU oracle (Section 2.1 problem statement) against things other
than itself: path enumeration straight from the definition, Floyd-Warshall,
closed forms, a hand-worked example and scipy's Dijkstra."""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle

INF = oracle.UNREACHABLE


# ---------------------------------------------------------------- brute force

def enumerate_paths_distance(g, src):
    """Definition of l_su (Section 2.1): min over s->u paths of the weight sum.
    With non-negative weights a shortest walk can be shortened to a simple path,
    so enumerating simple paths by DFS gives the exact minimum."""
    adj = [[] for _ in range(g.n)]
    for u in range(g.n):
        for e in range(g.off[u], g.off[u + 1]):
            adj[u].append((int(g.col[e]), int(g.w[e])))
    best = [None] * g.n
    on_path = [False] * g.n

    def dfs(u, length):
        if best[u] is None or length < best[u]:
            best[u] = length
        on_path[u] = True
        for v, w in adj[u]:
            if not on_path[v]:
                dfs(v, length + w)
        on_path[u] = False

    dfs(src, 0)
    return [INF if b is None else b for b in best]


def floyd_warshall(g):
    n = g.n
    D = [[None] * n for _ in range(n)]
    for u in range(n):
        D[u][u] = 0
        for e in range(g.off[u], g.off[u + 1]):
            v, w = int(g.col[e]), int(g.w[e])
            if D[u][v] is None or w < D[u][v]:
                D[u][v] = w
    for k in range(n):
        for i in range(n):
            if D[i][k] is None:
                continue
            for j in range(n):
                if D[k][j] is None:
                    continue
                c = D[i][k] + D[k][j]
                if D[i][j] is None or c < D[i][j]:
                    D[i][j] = c
    return [[INF if x is None else x for x in row] for row in D]


@pytest.mark.parametrize("wmin,wmax", [(0, 3), (1, 255), (0, 0)])
def test_dijkstra_matches_path_enumeration(wmin, wmax):
    rng = np.random.default_rng(1234 + wmax)
    for trial in range(400):
        n = int(rng.integers(1, 8))
        g = gg.random_small(n, int(rng.integers(0, 3 * n + 1)), wmax, rng, wmin=wmin)
        src = int(rng.integers(0, n))
        want = enumerate_paths_distance(g, src)
        assert oracle.dijkstra(g, src).tolist() == want, (trial, n)


def test_dijkstra_and_bellman_ford_match_floyd_warshall():
    rng = np.random.default_rng(99)
    for trial in range(300):
        n = int(rng.integers(1, 13))
        wmax = int(rng.choice([3, 255]))
        g = gg.random_small(n, int(rng.integers(0, 4 * n + 1)), wmax, rng, wmin=0)
        fw = floyd_warshall(g)
        for src in range(n):
            d = oracle.dijkstra(g, src).tolist()
            assert d == fw[src], (trial, src)
            assert oracle.bellman_ford(g, src).tolist() == fw[src]


def test_dijkstra_matches_bellman_ford_many_tiny_graphs():
    rng = np.random.default_rng(7)
    for trial in range(10000):
        n = int(rng.integers(1, 13))
        wmax = 3 if trial % 2 else 255
        g = gg.random_small(n, int(rng.integers(0, 3 * n + 1)), wmax, rng, wmin=0)
        src = int(rng.integers(0, n))
        assert np.array_equal(oracle.dijkstra(g, src), oracle.bellman_ford(g, src)), trial


# ---------------------------------------------------------------- closed forms

def test_uniform_weight_grid_is_scaled_manhattan():
    R, C, c = 23, 31, 7
    g = gg.grid(R, C, 0.0, wmax=255, seed=5)
    g.w[:] = c
    for r0, c0 in [(0, 0), (11, 17), (22, 30)]:
        src = r0 * C + c0
        rr, cc = np.divmod(np.arange(R * C), C)
        want = c * (np.abs(rr - r0) + np.abs(cc - c0))
        assert np.array_equal(oracle.dijkstra(g, src), want.astype(np.uint32))


def test_path_is_prefix_sums():
    rng = np.random.default_rng(3)
    n = 500
    w = rng.integers(0, 1000, n - 1)
    g = gg.from_edges(n, np.arange(n - 1), np.arange(1, n), w)
    d = oracle.dijkstra(g, 0)
    assert np.array_equal(d, np.concatenate([[0], np.cumsum(w)]).astype(np.uint32))
    # the directed path is not reachable backwards
    d = oracle.dijkstra(g, 250)
    assert (d[:250] == INF).all() and d[250] == 0


def test_star_distances_are_edge_weights():
    rng = np.random.default_rng(4)
    n = 300
    w = rng.integers(1, 256, n - 1)
    leaves = np.arange(1, n)
    g = gg.from_edges(n, np.concatenate([np.zeros(n - 1, int), leaves]),
                      np.concatenate([leaves, np.zeros(n - 1, int)]), np.concatenate([w, w]))
    assert np.array_equal(oracle.dijkstra(g, 0)[1:], w.astype(np.uint32))
    d = oracle.dijkstra(g, 5)   # leaf 5 -> centre -> other leaves
    assert d[0] == w[4] and np.array_equal(d[1:], np.where(leaves == 5, 0, w[4] + w).astype(np.uint32))


def test_zero_weights_give_zero_on_reachable_set():
    g = gg.rmat(10, 4, seed=3)
    g.w[:] = 0
    src = gg.max_degree_vertex(g)
    d = oracle.dijkstra(g, src)
    # reachability by plain BFS
    seen = np.zeros(g.n, bool)
    seen[src] = True
    frontier = [src]
    while frontier:
        nxt = []
        for u in frontier:
            for v in g.col[g.off[u]:g.off[u + 1]]:
                if not seen[v]:
                    seen[v] = True
                    nxt.append(int(v))
        frontier = nxt
    assert np.array_equal(d, np.where(seen, 0, INF).astype(np.uint32))


def test_isolated_source():
    g = gg.from_edges(4, [1, 2], [2, 3], [5, 5])
    assert oracle.dijkstra(g, 0).tolist() == [0, INF, INF, INF]


# ---------------------------------------------------------------- overflow

def test_overflow_boundary():
    big = 2**31
    # 2^31 + (2^31 - 2) = 2^32 - 2 : largest representable finite distance
    g = gg.from_edges(3, [0, 1], [1, 2], [big, big - 2])
    assert oracle.dijkstra(g, 0).tolist() == [0, big, 2**32 - 2]
    assert oracle.bellman_ford(g, 0).tolist() == [0, big, 2**32 - 2]
    # 2^32 - 1 collides with the sentinel: overflow
    g = gg.from_edges(3, [0, 1], [1, 2], [big, big - 1])
    with pytest.raises(oracle.OracleError) as ei:
        oracle.dijkstra(g, 0)
    assert ei.value.code == oracle.ERR_DISTANCE_OVERFLOW
    with pytest.raises(oracle.OracleError):
        oracle.bellman_ford(g, 0)
    # a longer but non-shortest route that would overflow is harmless
    g = gg.from_edges(3, [0, 1, 0], [1, 2, 2], [big, big, 5])
    assert oracle.dijkstra(g, 0).tolist() == [0, big, 5]


def test_invalid_arguments():
    g = gg.from_edges(3, [0], [1], [1])
    with pytest.raises(oracle.OracleError):
        oracle.dijkstra(g, 3)
    with pytest.raises(oracle.OracleError):
        oracle.dijkstra(g, -1)


# ---------------------------------------------------------------- worked example

def test_redundant_wavefront_example(golden):
    n, src, edges, expect = golden("redundant_wavefront.txt")
    u, v, w = zip(*edges)
    g = gg.from_edges(n, u, v, w)
    d = oracle.dijkstra(g, src)
    assert {i: int(d[i]) for i in range(n)} == expect
    # the three routes to v obey the inequality printed in the paper
    assert 10 > 3 + 6 > 1 + 2 + 3
    assert oracle.bellman_ford(g, src).tolist() == d.tolist()
    assert oracle.certificate(g, src, d)[0] == oracle.OK


# ---------------------------------------------------------------- library cross-check

@pytest.mark.parametrize("kind", ["grid", "road", "rmat", "uniform"])
def test_dijkstra_matches_scipy(kind):
    sp = pytest.importorskip("scipy.sparse")
    csgraph = pytest.importorskip("scipy.sparse.csgraph")
    if kind == "grid":
        g = gg.grid(64, 80, 0.0, seed=11)
    elif kind == "road":
        g = gg.grid(128, 128, 0.3, seed=12)
    elif kind == "rmat":
        g = gg.rmat(13, 8, seed=13)
    else:
        g = gg.uniform(5000, 40000, seed=14)
    # generators produce no parallel edges and weights >= 1, so the sparse
    # matrix holds exactly the edge set (scipy would sum duplicates)
    A = sp.csr_matrix((g.w.astype(np.float64), g.col, g.off), shape=(g.n, g.n))
    rng = np.random.default_rng(0)
    for src in rng.choice(g.n, 4, replace=False):
        ref = csgraph.dijkstra(A, directed=True, indices=int(src))
        want = np.where(np.isinf(ref), INF, ref).astype(np.uint64)
        assert np.array_equal(oracle.dijkstra(g, int(src)).astype(np.uint64), want)


# ---------------------------------------------------------------- certificate

def test_certificate_accepts_correct_and_rejects_corruptions():
    rng = np.random.default_rng(21)
    rejected = 0
    for trial in range(300):
        n = int(rng.integers(2, 30))
        g = gg.random_small(n, int(rng.integers(n, 4 * n)), int(rng.choice([3, 255])), rng, wmin=0)
        src = int(rng.integers(0, n))
        d = oracle.dijkstra(g, src)
        assert oracle.certificate(g, src, d)[0] == oracle.OK
        for kind in ("up", "down", "to_inf", "to_finite", "source"):
            bad = d.copy()
            fin = np.nonzero((d != INF) & (np.arange(n) != src))[0]
            unr = np.nonzero(d == INF)[0]
            if kind == "up" and fin.size:
                bad[rng.choice(fin)] += 1
            elif kind == "down" and fin.size and (d[fin] > 0).any():
                bad[rng.choice(fin[d[fin] > 0])] -= 1
            elif kind == "to_inf" and fin.size:
                bad[rng.choice(fin)] = INF
            elif kind == "to_finite" and unr.size:
                bad[rng.choice(unr)] = int(rng.integers(0, 100))
            elif kind == "source":
                bad[src] = 1
            else:
                continue
            code = oracle.certificate(g, src, bad)[0]
            assert code != oracle.OK, (trial, kind)
            rejected += 1
    assert rejected > 800


def test_certificate_rejects_self_supporting_zero_cycle():
    # s -> a (5), a <-> b with weight 0. Claiming a = b = 3 satisfies every edge
    # inequality and gives both a tight in-edge, but no tight path from s.
    g = gg.from_edges(3, [0, 1, 2], [1, 2, 1], [5, 0, 0])
    assert oracle.certificate(g, 0, np.array([0, 5, 5], np.uint32))[0] == oracle.OK
    rc, where, _ = oracle.certificate(g, 0, np.array([0, 3, 3], np.uint32))
    assert rc == oracle.CERT_UNSUPPORTED and where in (1, 2)


def test_certificate_flags_overflowed_vertex():
    big = 2**31
    g = gg.from_edges(3, [0, 1], [1, 2], [big, big])
    d = oracle.dijkstra(g, 0, allow_overflow=True)
    assert d.tolist() == [0, big, INF]
    assert oracle.certificate(g, 0, d)[0] == oracle.CERT_EDGE_VIOLATED


def test_certificate_depth_is_fewest_hop_depth():
    R, C = 9, 13
    g = gg.grid(R, C, 0.0, seed=1)
    g.w[:] = 1
    d = oracle.dijkstra(g, 0)
    assert oracle.certificate(g, 0, d) == (oracle.OK, -1, (R - 1) + (C - 1))


def test_reach_stats():
    g = gg.from_edges(5, [0, 0, 1, 3, 3], [1, 2, 2, 4, 0], [1, 1, 1, 1, 1])
    d = oracle.dijkstra(g, 0)
    assert oracle.reach_stats(g, d) == (3, 3)


# ---------------------------------------------------------------- BFS (Section 5.7)

def test_bfs_grid_is_manhattan_distance():
    """Closed form: on a full R x C grid, the fewest hops are |dr| + |dc|."""
    R, C = 23, 31
    g = gg.grid(R, C, 0.0, seed=4)
    src = 7 * C + 11
    lv = oracle.bfs(g, src)
    r, c = np.divmod(np.arange(R * C), C)
    assert np.array_equal(lv, np.abs(r - 7) + np.abs(c - 11))


def test_bfs_path_and_unreachable():
    n = 50
    g = gg.from_edges(n, np.arange(n - 1), np.arange(1, n), np.full(n - 1, 200))
    assert np.array_equal(oracle.bfs(g, 0), np.arange(n))
    lv = oracle.bfs(g, 10)  # edges point forward only
    assert (lv[:10] == oracle.UNREACHABLE).all() and np.array_equal(lv[10:], np.arange(n - 10))


def test_bfs_equals_dijkstra_with_unit_weights():
    """Independent reference: Dijkstra on the same graph with every weight 1."""
    rng = np.random.default_rng(17)
    for trial in range(60):
        n = int(rng.integers(2, 40))
        g = gg.random_small(n, int(rng.integers(0, 4 * n)), int(rng.integers(0, 2**31)), rng, wmin=0)
        unit = gg.Csr(g.n, g.off, g.col, np.ones_like(g.w))
        s = int(rng.integers(0, n))
        assert np.array_equal(oracle.bfs(g, s), oracle.dijkstra(unit, s)), trial


def test_bfs_matches_scipy_unweighted():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    g = gg.rmat(10, 8, seed=9)
    s = gg.max_degree_vertex(g)
    a = csr_matrix((np.ones(g.m), g.col, g.off), shape=(g.n, g.n))
    ref = shortest_path(a, unweighted=True, indices=s)
    want = np.where(np.isinf(ref), oracle.UNREACHABLE, ref).astype(np.uint32)
    assert np.array_equal(oracle.bfs(g, s), want)
