"""The library's HIP kernel source executed on the CPU (one host thread per
lane, cross-lane builtins as barrier exchanges; see tests/simt), checked
against the oracle. Runs without a GPU; catches logic errors in the queue
protocol, lane divergence around cross-lane operations and out-of-range
indices (every edge and vertex index is bounds-checked in this build)."""
import ctypes
import os
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from check_count import check_count as _check_count

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# knobs: l0_rows, l1_type, l2_type, l1_cap, l1_wb, delta1, d2_log2, bmax, bnum,
#        th_v, th_hub, hub_chunk, nb_log2, hub_cap, timeout_ms, relax_mode, unit_w[, pnum]
CFG = {
    "L0x2-L1V-L2V": [2, 1, 0, 1024, 64, 256, 7, 32, 4, 32, 0, 2048, 10, 1, 60000, 0, 0],
    "L0off-L1none-L2V": [0, 0, 0, 1024, 64, 256, 7, 32, 4, 32, 0, 2048, 10, 1, 60000, 0, 0],
    "L0x4-L1V-wb4-tiny": [4, 1, 0, 64, 4, 256, 7, 32, 4, 32, 0, 2048, 4, 1, 60000, 0, 0],
    "L1NF-L2V": [1, 2, 0, 1024, 0, 64, 7, 32, 4, 32, 0, 2048, 10, 1, 60000, 0, 0],
    "L1FQ-L2V": [1, 3, 0, 1024, 0, 64, 7, 32, 4, 32, 0, 2048, 10, 1, 60000, 0, 0],
    "L1NF-L2DQ": [1, 2, 1, 1024, 0, 32, 5, 32, 2, 32, 0, 2048, 8, 1, 60000, 0, 0],
    "L1FQ-L2DQ-hub": [1, 3, 1, 1024, 0, 128, 8, 8, 8, 32, 128, 128, 8, 256, 60000, 0, 0],
    "L1V-L2V-hub64": [2, 1, 0, 1024, 64, 256, 7, 32, 4, 8, 64, 64, 10, 256, 60000, 0, 0],
    "L0off-L1NF-L2V-atomic": [0, 2, 0, 256, 0, 64, 7, 32, 4, 32, 0, 2048, 10, 1, 60000, 1, 0],
    "L0x1-L1SLF-L2V": [1, 4, 0, 128, 0, 64, 7, 32, 4, 32, 0, 2048, 10, 1, 60000, 0, 0],
    "L0x1-L1SLF-L2DQ-hub": [1, 4, 1, 256, 0, 64, 6, 16, 1, 16, 128, 128, 8, 256, 60000, 0, 0],
    # priority queues (Section 4.2): alone, under L0 + L1, and as a multi-queue
    "L1none-L2PQ": [0, 0, 2, 1024, 0, 64, 7, 32, 4, 32, 0, 2048, 8, 1, 60000, 0, 0, 1],
    "L0x1-L1NF-L2PQ": [1, 2, 2, 256, 0, 64, 7, 32, 4, 32, 0, 2048, 8, 1, 60000, 0, 0, 1],
    "L0x1-L1V-L2MPQ3-hub": [1, 1, 2, 256, 16, 64, 7, 32, 4, 16, 128, 128, 6, 256, 60000, 0, 0, 3],
}


def _knobs(k):
    """Knob array with the priority-queue count appended when absent (1)."""
    k = list(k)
    return k + [1] * (18 - len(k))


@pytest.fixture(scope="module")
def sim():
    sys.path.insert(0, os.path.join(HERE, "simt"))
    import build_sim
    lib = ctypes.CDLL(build_sim.build(os.path.join(ROOT, "_build", "simt")))
    lib.sim_sssp.restype = ctypes.c_int
    return lib


def run(lib, csr, src, knobs, nwg=8):
    off = csr.off32()
    col = np.ascontiguousarray(csr.col, np.int32)
    w = np.ascontiguousarray(csr.w, np.uint32)
    dist = np.zeros(csr.n, np.uint32)
    k = np.array(_knobs(knobs), np.uint32)
    stats = np.zeros(16, np.uint64)
    status = np.zeros(4, np.uint32)
    vp = ctypes.c_void_p
    lib.sim_sssp(ctypes.c_int32(csr.n), vp(off.ctypes.data), vp(col.ctypes.data), vp(w.ctypes.data),
                 ctypes.c_uint32(src), vp(dist.ctypes.data), vp(k.ctypes.data), ctypes.c_uint32(nwg),
                 ctypes.c_uint32(64), vp(stats.ctypes.data), vp(status.ctypes.data))
    return dist, status, stats


GRAPHS = {
    "grid16": lambda: (gg.grid(16, 16, 0.0, seed=1), 0),
    "road24": lambda: (gg.grid(24, 20, 0.1, seed=2), 77),
    "rmat9": lambda: (lambda g: (g, gg.max_degree_vertex(g)))(gg.rmat(9, 8, seed=3)),
    # two hubs of 1500 leaves, joined: long rows swept by one wave (re-checked every 1024 edges)
    "hubs": lambda: (_hubs(), 0),
}


def _hubs():
    rng = np.random.default_rng(7)
    a = np.arange(2, 1502)
    b = np.arange(1502, 3002)
    src = np.concatenate([np.zeros(1500, int), a, np.ones(1500, int), b, [0, 1]] + [a[:700]])
    dst = np.concatenate([a, np.zeros(1500, int), b, np.ones(1500, int), [1, 0]] + [b[:700]])
    w = rng.integers(1, 256, src.size)
    return gg.from_edges(3002, src, dst, w)


@pytest.mark.parametrize("cfg", list(CFG))
@pytest.mark.parametrize("graph", list(GRAPHS))
def test_kernel_on_cpu_matches_oracle(sim, graph, cfg):
    csr, src = GRAPHS[graph]()
    dist, status, stats = run(sim, csr, src, CFG[cfg])
    assert status[0] == 0, f"device status {status[0]}"
    assert np.array_equal(dist, oracle.dijkstra(csr, src))
    # delayed counting balanced: every reserved block was consumed
    assert status[2] >= 1


@pytest.mark.parametrize("cfg", ["L0x2-L1V-L2V", "L1FQ-L2DQ-hub", "L0x1-L1NF-L2PQ"])
@pytest.mark.parametrize("nslots,want,nwg", [(2, 3, 6), (3, 8, 6), (1, 5, 16)])
def test_server_kernel_on_cpu_matches_oracle(sim, cfg, nslots, want, nwg):
    """Slot protocol of the resident server kernel: queries join (one ticket
    each; waves that lose the race to a full slot count past want and stay
    out), run next to each other, close, and the last wave out reports
    completion; each result equals the oracle's. Queries share the grid when
    want < nwg; with one slot and 16 waves for 5 places most joins lose."""
    csr, _ = GRAPHS["road24"]()
    srcs = np.array([0, 77, 479, 200, 13, 77, 301], np.uint32)
    nq = len(srcs)
    off = csr.off32()
    col = np.ascontiguousarray(csr.col, np.int32)
    w = np.ascontiguousarray(csr.w, np.uint32)
    dist = np.zeros((nq, csr.n), np.uint32)
    status = np.full(nq, 0xFFFF, np.uint32)
    k = np.array(_knobs(CFG[cfg]), np.uint32)
    vp = ctypes.c_void_p
    sim.sim_server.restype = ctypes.c_int
    rc = sim.sim_server(ctypes.c_int32(csr.n), vp(off.ctypes.data), vp(col.ctypes.data), vp(w.ctypes.data),
                        ctypes.c_int32(nq), vp(srcs.ctypes.data), vp(dist.ctypes.data), vp(k.ctypes.data),
                        ctypes.c_uint32(nwg), ctypes.c_int32(nslots), ctypes.c_uint32(want),
                        vp(status.ctypes.data))
    assert rc == 0, "not every query completed"
    assert (status == 0).all(), status
    for i, s in enumerate(srcs):
        assert np.array_equal(dist[i], oracle.dijkstra(csr, int(s))), i


@pytest.mark.parametrize("cfg", ["L0x2-L1V-L2V", "L1NF-L2DQ", "L0x1-L1SLF-L2V", "L1none-L2PQ"])
@pytest.mark.parametrize("graph", ["road24", "rmat9"])
def test_bfs_mode_on_cpu_matches_oracle(sim, graph, cfg):
    """Unit-weight mode (breadth-first levels, Section 5.7)."""
    csr, src = GRAPHS[graph]()
    k = list(CFG[cfg])
    k[16] = 1
    dist, status, _ = run(sim, csr, src, k)
    assert status[0] == 0
    assert np.array_equal(dist, oracle.bfs(csr, src))


# ------------------------------------------------------------ optimality check

def _sim_check(lib, csr, src, d, nwg):
    off = csr.off32()
    col = np.ascontiguousarray(csr.col, np.int32)
    w = np.ascontiguousarray(csr.w, np.uint32)
    d = np.ascontiguousarray(d, np.uint32)
    bad = ctypes.c_uint64()
    vp = ctypes.c_void_p
    lib.sim_check(ctypes.c_int32(csr.n), vp(off.ctypes.data), vp(col.ctypes.data), vp(w.ctypes.data),
                  ctypes.c_uint32(src), vp(d.ctypes.data), ctypes.c_uint32(nwg), ctypes.byref(bad))
    return int(bad.value)


def _check_graphs():
    rng = np.random.default_rng(5)
    # a star whose centre row spans three 4096-edge slices, plus isolated vertices between rows
    n = 9000
    centre = np.zeros(8500, int)
    leaves = rng.choice(np.arange(1, n), 8500, replace=False)
    star = gg.from_edges(n, np.concatenate([centre, leaves]), np.concatenate([leaves, centre]),
                         rng.integers(1, 40, 17000))
    return {"grid16": (gg.grid(16, 16, 0.0, seed=1), 0), "road24": (gg.grid(24, 20, 0.1, seed=2), 77),
            "rmat10": (lambda g: (g, gg.max_degree_vertex(g)))(gg.rmat(10, 8, seed=3)),
            "star": (star, 0), "hubs": (_hubs(), 0),
            "edgeless": (gg.from_edges(5, [], [], []), 2)}


@pytest.mark.parametrize("graph", ["grid16", "road24", "rmat10", "star", "hubs", "edgeless"])
def test_check_kernel_on_cpu(sim, graph):
    """The check accepts the oracle's distances and rejects perturbed vectors;
    its count equals the conditions counted directly, its verdict equals the
    oracle's certificate."""
    csr, src = _check_graphs()[graph]
    want = oracle.dijkstra(csr, src)
    rng = np.random.default_rng(11)
    reach = np.nonzero(want != oracle.UNREACHABLE)[0]
    unreach = np.nonzero(want == oracle.UNREACHABLE)[0]
    cases = [want.copy()]
    for _ in range(1):
        if reach.size > 1:
            for delta in (-1, 1):
                d = want.copy()
                v = int(rng.choice(reach[reach != src]))
                d[v] = np.uint32(int(d[v]) + delta)
                cases.append(d)
            d = want.copy()
            d[int(rng.choice(reach[reach != src]))] = oracle.UNREACHABLE
            cases.append(d)
        if unreach.size:
            d = want.copy()
            d[int(rng.choice(unreach))] = 5
            cases.append(d)
    d = want.copy()
    d[src] = 1
    cases.append(d)
    for i, d in enumerate(cases):
        for nwg in ((1, 3) if i == 0 else (3,)):
            got = _sim_check(sim, csr, src, d, nwg)
            assert got == _check_count(csr, src, d), (i, nwg)
            code, _, _ = oracle.certificate(csr, src, d)
            assert (got == 0) == (code == 0), (i, nwg, got, code)


# ------------------------------------------------------------ queue-unit example

@pytest.mark.parametrize("l1_type,delta1,read,left,l2", [
    # vector: FIFO, the first two read are {5, 1}
    (1, 64, [5, 1, 2], [], []),
    # near-far: NF = min of the first batch + delta1 = 3, so {1, 2} near and 5 kept far
    (2, 2, [1, 2], [5], []),
    # filter: F = 3, so {1, 2} kept and 5 sent to the global level
    (3, 3, [1, 2], [], [5]),
    # Small-Label-First deque: 5; 1 in front of 5; 2 behind: [1, 5, 2]
    (4, 64, [1, 5, 2], [], []),
])
def test_queue_unit_example(sim, l1_type, delta1, read, left, l2):
    """Section 3.4's queue example (its figure is missing from the text, so
    this pins our reading): distances 5, 1, 2 written one at a time to a
    wave's L1, then one L1 read, for each L1 policy of the kernel."""
    rd, lf, l2d = (np.zeros(64, np.uint32) for _ in range(3))
    nr, nl, n2 = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    vp = ctypes.c_void_p
    sim.sim_l1_example(ctypes.c_uint32(l1_type), ctypes.c_uint32(delta1), vp(rd.ctypes.data), ctypes.byref(nr),
                       vp(lf.ctypes.data), ctypes.byref(nl), vp(l2d.ctypes.data), ctypes.byref(n2))
    assert list(rd[:nr.value]) == read
    assert list(lf[:nl.value]) == left
    assert list(l2d[:n2.value]) == l2


# ------------------------------------------------------------ priority queues alone

def _sim_pq(lib, nwaves, pnum, nb_log2, rounds, pop_every, dmax, seed):
    cap = nwaves * rounds * 64
    ins = np.zeros(cap, np.uint64)
    out = np.zeros(cap, np.uint64)
    nin, nout, unsorted, disorder = (ctypes.c_uint32() for _ in range(4))
    status = np.zeros(3, np.uint32)
    vp = ctypes.c_void_p
    lib.sim_pq(ctypes.c_uint32(nwaves), ctypes.c_uint32(pnum), ctypes.c_uint32(nb_log2), ctypes.c_uint32(rounds),
               ctypes.c_uint32(pop_every), ctypes.c_uint32(dmax), ctypes.c_uint64(seed), vp(ins.ctypes.data),
               ctypes.byref(nin), vp(out.ctypes.data), ctypes.byref(nout), ctypes.byref(unsorted),
               ctypes.byref(disorder), vp(status.ctypes.data))
    return ins[:nin.value], out[:nout.value], unsorted.value, disorder.value, status


@pytest.mark.parametrize("dmax", [1000, 7])
def test_priority_queue_single_wave_is_exact(sim, dmax):
    """One wave writes 24 batches of 1..64 elements, then takes everything:
    the batched heap returns every element once, each taken batch ascending,
    and the whole sequence in ascending distance order (an exact priority
    queue; dmax = 7 makes most keys tie on distance)."""
    ins, out, unsorted, disorder, st = _sim_pq(sim, 1, 1, 5, 24, 0, dmax, 11)
    assert st[0] == 0 and st[2] == 0
    assert st[1] == ins.size
    assert np.array_equal(np.sort(ins), np.sort(out))
    assert unsorted == 0 and disorder == 0


@pytest.mark.parametrize("nwaves,pnum,pop_every", [(6, 1, 2), (6, 1, 1), (8, 3, 2), (5, 4, 3)])
def test_priority_queues_concurrent_conserve_elements(sim, nwaves, pnum, pop_every):
    """Several waves write and take concurrently (per-node locks, hand-over-hand
    insertion, sinking deletions; pnum > 1 is the multi-queue): no element is
    lost or duplicated, every taken batch is ascending, the queues end empty
    and the termination count (pq_in) equals the elements written."""
    ins, out, unsorted, _, st = _sim_pq(sim, nwaves, pnum, 7, 30, pop_every, 100000, 5 + nwaves)
    assert st[0] == 0, f"device status {st[0]}"
    assert st[1] == ins.size and st[2] == 0
    assert np.array_equal(np.sort(ins), np.sort(out))
    assert unsorted == 0


def test_priority_queue_capacity_is_reported(sim):
    """More full batches than the heap has nodes: the write reports the
    capacity status (the library then retries with a larger heap)."""
    _, _, _, _, st = _sim_pq(sim, 1, 1, 3, 24, 0, 1000, 3)
    assert st[0] == 1
