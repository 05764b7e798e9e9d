"""Seeded generator: reproducibility and the structural promises each graph
family makes (counts, symmetry, no self-loops or duplicates, weight range)."""
import hashlib

import numpy as np
import pytest

import graphgen as gg


def digest(g):
    h = hashlib.sha256()
    for a in (g.off, g.col, g.w):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def edge_weights(g):
    src = np.repeat(np.arange(g.n), g.degrees())
    return {(int(u), int(v)): int(w) for u, v, w in zip(src, g.col, g.w)}


def check_rows_sorted_unique(g):
    for u in range(g.n):
        row = g.col[g.off[u]:g.off[u + 1]]
        assert (np.diff(row) > 0).all(), u


def test_same_seed_same_graph_and_thread_independence():
    a = gg.rmat(12, 16, seed=77)
    old = gg.set_threads(1)
    try:
        b = gg.rmat(12, 16, seed=77)
    finally:
        gg.set_threads(old)
    c = gg.rmat(12, 16, seed=78)
    assert digest(a) == digest(b) != digest(c)
    assert digest(gg.grid(64, 64, 0.05, seed=3)) == digest(gg.grid(64, 64, 0.05, seed=3))


def test_grid_counts_and_structure():
    R, C = 37, 53
    g = gg.grid(R, C, 0.0, seed=2)
    assert g.n == R * C and g.m == 2 * (R * (C - 1) + C * (R - 1))
    check_rows_sorted_unique(g)
    ew = edge_weights(g)
    for (u, v), w in ew.items():
        ru, cu = divmod(u, C)
        rv, cv = divmod(v, C)
        assert abs(ru - rv) + abs(cu - cv) == 1
        assert ew[(v, u)] == w and 1 <= w <= 255
    assert g.degrees().max() == 4


def test_grid_drop_rate_and_symmetry():
    g = gg.grid(300, 300, 0.05, seed=9)
    full = 2 * (300 * 299 * 2)
    assert abs(g.m / full - 0.95) < 0.005
    ew = edge_weights(g)
    assert all(ew[(v, u)] == w for (u, v), w in ew.items())


def test_rmat_structure():
    g = gg.rmat(11, 16, seed=5)
    check_rows_sorted_unique(g)
    src = np.repeat(np.arange(g.n), g.degrees())
    assert not (src == g.col).any()
    ew = edge_weights(g)
    assert all(ew[(v, u)] == w for (u, v), w in ew.items())
    assert g.w.min() >= 1 and g.w.max() <= 255
    # skewed degrees: the hub is far above the mean
    assert g.degrees().max() > 20 * g.degrees().mean()


def test_rmat_permutation_is_a_relabelling():
    a = gg.rmat(10, 8, permute=False, seed=4)
    b = gg.rmat(10, 8, permute=True, seed=4)
    assert a.m == b.m
    assert np.array_equal(np.sort(a.degrees()), np.sort(b.degrees()))
    assert not np.array_equal(a.degrees(), b.degrees())


def test_uniform_structure():
    g = gg.uniform(4096, 40000, wmax=65535, seed=6)
    check_rows_sorted_unique(g)
    src = np.repeat(np.arange(g.n), g.degrees())
    assert not (src == g.col).any()
    assert 39000 < g.m <= 40000
    assert g.w.min() >= 1 and g.w.max() <= 65535 and g.w.max() > 60000


def test_sources():
    g = gg.rmat(10, 8, seed=4)
    s = gg.max_degree_vertex(g)
    assert g.degrees()[s] == g.degrees().max()
    assert (g.degrees()[:s] < g.degrees()[s]).all()
    srcs = gg.sample_sources(g, 50, seed=1)
    assert len(set(srcs.tolist())) == 50 and (g.degrees()[srcs] > 0).all()
    assert np.array_equal(srcs, gg.sample_sources(g, 50, seed=1))


def test_from_edges_keeps_multi_edges_and_loops():
    g = gg.from_edges(3, [0, 0, 1, 1], [1, 1, 1, 2], [4, 2, 0, 7])
    assert g.m == 4 and g.off.tolist() == [0, 2, 4, 4]
    with pytest.raises(ValueError):
        gg.from_edges(3, [0], [3], [1])
