"""GPU tests of the paths the parity grid does not reach: the exact overflow
test's false alarm (a saturating candidate that is not a shortest path) in
the plain, batched and serving forms; the device watchdog; the refusal of
multi-wave workgroups; batches whose queue layout changes between launches;
concurrent solves from two host threads on two streams; a server whose
graphs are all power-law (register-bound residency); batches and servers
that mix priority-queue queries (their own kernel variant) with ring queries;
and plain solves on a power-law graph's degree-ordered copy.
Every result is compared with the oracle element by element (integer
arithmetic, tolerance 0)."""
import sys
import threading
import time

import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mlmq():
    import paper_2602_10080_amd as mlmq
    return mlmq


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _false_alarm():
    # 0 -> 1 (2^31), 1 -> 2 (2^31), 0 -> 2 (5): expanding vertex 1 yields the
    # candidate 2^32 for vertex 2, which saturates and raises the overflow
    # flag, but the true distances 0, 2^31, 5 all fit (Section 2.1's problem
    # with uint32 distances; the graph is not overflow-safe, so the exact test
    # runs and must clear the alarm)
    return gg.from_edges(3, [0, 1, 0], [1, 2, 2], [2**31, 2**31, 5])


def test_false_alarm_plain():
    mlmq = _mlmq()
    csr = _false_alarm()
    g = mlmq.Graph.from_csr(csr)
    want = oracle.dijkstra(csr, 0)
    assert want.tolist() == [0, 2**31, 5]
    for kw in ({}, dict(l0_rows=0, l1_type=0, l2_type=0, th_hub=0), dict(l1_type=2, l2_type=1, th_hub=0)):
        out = mlmq.sssp(g, 0, config=mlmq.default_config(**kw) if kw else None)
        torch.cuda.synchronize()
        assert mlmq.to_numpy(out).tolist() == want.tolist(), kw
    host = np.empty(3, np.uint32)
    mlmq.sssp(g, 0, out=host)
    assert host.tolist() == want.tolist()
    g.close()


def test_false_alarm_batch():
    mlmq = _mlmq()
    fa = _false_alarm()
    grid = gg.grid(64, 64, 0.05, seed=1)
    gf, gd = mlmq.Graph.from_csr(fa), mlmq.Graph.from_csr(grid)
    graphs = [gf, gd, gf, gd]
    csrs = [fa, grid, fa, grid]
    srcs = [0, 7, 0, 100]
    outs, status = mlmq.sssp_batch(graphs, srcs)
    torch.cuda.synchronize()
    assert status == [0] * 4
    for c, s, o in zip(csrs, srcs, outs):
        assert np.array_equal(mlmq.to_numpy(o), oracle.dijkstra(c, s))


def test_false_alarm_server():
    mlmq = _mlmq()
    fa = _false_alarm()
    grid = gg.grid(64, 64, 0.05, seed=1)
    graphs = [mlmq.Graph.from_csr(fa), mlmq.Graph.from_csr(grid)]
    outs = [mlmq.new_dist(3), mlmq.new_dist(grid.n), mlmq.new_dist(3)]
    torch.cuda.synchronize()
    srv = mlmq.Server(graphs, mem_budget_bytes=1 << 28, max_slots=4)
    try:
        t = [srv.submit(0, 0, outs[0]), srv.submit(1, 5, outs[1]), srv.submit(0, 0, outs[2])]
        status = [srv.wait(x, 30000) for x in t]
    finally:
        srv.close()
    assert status == [0, 0, 0]
    assert mlmq.to_numpy(outs[0]).tolist() == [0, 2**31, 5]
    assert mlmq.to_numpy(outs[2]).tolist() == [0, 2**31, 5]
    assert np.array_equal(mlmq.to_numpy(outs[1]), oracle.dijkstra(grid, 5))


def test_device_watchdog_then_clean_solve():
    """A 1 ms device deadline on a solve that takes several: every wave leaves
    on its own bounded wait, the call reports MLMQ_ERR_TIMEOUT, and the next
    solve on the same graph (queue memory from the same pool) is exact."""
    mlmq = _mlmq()
    csr = gg.rmat(20, 16, seed=1)
    src = gg.max_degree_vertex(csr)
    g = mlmq.Graph.from_csr(csr)
    out = mlmq.new_dist(csr.n)
    _say(f"[watchdog] rmat20 n={csr.n} m={csr.m} timeout 1 ms")
    t0 = time.perf_counter()
    with pytest.raises(mlmq.MlmqError) as ei:
        mlmq.sssp(g, src, out=out, config=g.config().copy(timeout_ms=1, max_retries=0))
    took = time.perf_counter() - t0
    _say(f"[watchdog] {ei.value} after {took * 1e3:.1f} ms")
    assert ei.value.code == mlmq.ERR_TIMEOUT
    assert took < 2.0  # the device deadline, not the host's (timeout + 3 s)
    mlmq.sssp(g, src, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(mlmq.to_numpy(out), oracle.dijkstra(csr, src))
    g.close()


def test_multiwave_workgroups_refused():
    """Only one-wave workgroups exist (L1 private to its wave); any other
    size is refused before a launch."""
    mlmq = _mlmq()
    csr = gg.grid(16, 16, 0.0, seed=1)
    g = mlmq.Graph.from_csr(csr)
    for wg in (128, 256, 32):
        with pytest.raises(mlmq.MlmqError) as ei:
            mlmq.sssp(g, 0, config=mlmq.default_config(wg_size=wg))
        assert ei.value.code == mlmq.ERR_INVALID_ARG and "wg_size" in str(ei.value)
    out = mlmq.sssp(g, 0)
    torch.cuda.synchronize()
    assert np.array_equal(mlmq.to_numpy(out), oracle.dijkstra(csr, 0))
    g.close()


def test_batch_layout_changes_between_launches():
    """Two batches with the same query count whose queue memory differs in
    layout ([A, A, B] then [A, B, B] with different plan sizes): the second
    launch must not replay the first one's captured arguments."""
    mlmq = _mlmq()
    a = gg.grid(256, 256, 0.05, seed=41)  # 2n FIFO elements > the 64 Ki minimum
    b = gg.rmat(12, 8, seed=3)
    ga, gb = mlmq.Graph.from_csr(a), mlmq.Graph.from_csr(b)
    for rep, mix in enumerate(([0, 0, 1], [0, 1, 1], [1, 1, 0], [0, 0, 1])):
        graphs = [(ga, gb)[k] for k in mix]
        csrs = [(a, b)[k] for k in mix]
        srcs = [(rep * 977 + 13 * i) % c.n for i, c in enumerate(csrs)]
        _say(f"[batch-layout] rep={rep} mix={mix} srcs={srcs}")
        outs, status = mlmq.sssp_batch(graphs, srcs)
        torch.cuda.synchronize()
        assert status == [0, 0, 0]
        for c, s, o in zip(csrs, srcs, outs):
            assert np.array_equal(mlmq.to_numpy(o), oracle.dijkstra(c, s)), (rep, s)


def test_two_threads_two_streams():
    """Calls from two host threads on two streams at once: each result is the
    oracle's."""
    mlmq = _mlmq()
    road = gg.grid(300, 300, 0.05, seed=5)
    pl = gg.rmat(16, 16, seed=6)
    gr, gp = mlmq.Graph.from_csr(road), mlmq.Graph.from_csr(pl)
    jobs = {"road": (gr, road, [0, 150 * 300 + 150, 89999]), "rmat": (gp, pl, [gg.max_degree_vertex(pl), 1, 777])}
    want = {k: [oracle.dijkstra(c, s) for s in srcs] for k, (_, c, srcs) in jobs.items()}
    results, errors = {}, []

    def run(key):
        try:
            g, c, srcs = jobs[key]
            st = torch.cuda.Stream()
            outs = [torch.empty(c.n, dtype=torch.int32, device="cuda") for _ in srcs]
            for rep in range(3):
                for s, o in zip(srcs, outs):
                    mlmq.sssp(g, s, out=o, stream=st)
            st.synchronize()
            results[key] = [mlmq.to_numpy(o) for o in outs]
        except Exception as e:  # reported by the main thread
            errors.append(e)

    torch.cuda.synchronize()
    th = [threading.Thread(target=run, args=(k,)) for k in jobs]
    for t in th:
        t.start()
    for t in th:
        t.join(120)
    assert not errors, errors
    for k in jobs:
        for got, w in zip(results[k], want[k]):
            assert np.array_equal(got, w), k


def test_server_power_law_only_admission_latency():
    """A server over power-law graphs only, whose resident kernel is bounded by
    registers rather than LDS: admission kernels still find room beside it,
    so spread-out queries finish in milliseconds, and each equals the oracle."""
    mlmq = _mlmq()
    csrs = [gg.rmat(12, 16, seed=51), gg.rmat(14, 16, seed=52)]
    graphs = [mlmq.Graph.from_csr(c) for c in csrs]
    rng = np.random.default_rng(53)
    reqs = [(int(k), int(rng.integers(0, csrs[k].n))) for k in rng.integers(0, 2, 60)]
    outs = [mlmq.new_dist(csrs[k].n) for k, _ in reqs]
    torch.cuda.synchronize()
    srv = mlmq.Server(graphs, mem_budget_bytes=1 << 30, max_slots=16)
    lat = []
    try:
        tickets = []
        for i, ((k, s), o) in enumerate(zip(reqs, outs)):
            tickets.append(srv.submit(k, s, o))
            time.sleep(0.003 if i % 5 else 0.02)
        status = [srv.wait(t, 30000) for t in tickets]
        for t in tickets:
            a, b = srv.times(t)
            lat.append((b - a) / 1e6)
    finally:
        srv.close()
    lat = np.array(lat)
    _say(f"[server-pl] latency ms p50 {np.percentile(lat, 50):.2f} p99 {np.percentile(lat, 99):.2f} "
         f"max {lat.max():.2f}")
    assert status == [0] * len(reqs)
    for (k, s), o in zip(reqs, outs):
        assert np.array_equal(mlmq.to_numpy(o), oracle.dijkstra(csrs[k], s)), (k, s)
    assert np.percentile(lat, 99) < 100.0, lat.max()


def test_priority_queue_queries_in_batch_and_server():
    """Queries whose L2 is a priority queue (L2PQ) or a multi-queue (L2MPQ)
    mixed with ring queries in one batched launch and in one server: the
    library launches the kernel variant that holds the priority-queue code."""
    mlmq = _mlmq()
    road = gg.grid(128, 96, 0.05, seed=81)
    pl = gg.rmat(12, 8, seed=82)
    gr, gp = mlmq.Graph.from_csr(road), mlmq.Graph.from_csr(pl)
    pq1 = mlmq.default_config(l0_rows=1, l1_type=2, l2_type=2, pnum=1, delta1=64, th_hub=0)
    mpq = mlmq.default_config(l0_rows=1, l1_type=1, l2_type=2, pnum=8, th_hub=0)
    graphs = [gr, gp, gr, gp, gr, gp]
    csrs = [road, pl, road, pl, road, pl]
    cfgs = [pq1, mpq, None, None, mpq, pq1]
    srcs = [0, gg.max_degree_vertex(pl), 64 * 96 + 50, 7, 12287, 100]
    full = [c if c is not None else g.config() for c, g in zip(cfgs, graphs)]
    outs, status = mlmq.sssp_batch(graphs, srcs, configs=full)
    torch.cuda.synchronize()
    assert status == [0] * 6
    for c, s, o in zip(csrs, srcs, outs):
        assert np.array_equal(mlmq.to_numpy(o), oracle.dijkstra(c, s)), s
    outs = [mlmq.new_dist(c.n) for c in csrs]
    torch.cuda.synchronize()
    srv = mlmq.Server([gr, gp], mem_budget_bytes=1 << 28, max_slots=4, config=mpq)
    try:
        t = [srv.submit(0 if c is road else 1, s, o) for c, s, o in zip(csrs, srcs, outs)]
        st = [srv.wait(x, 30000) for x in t]
    finally:
        srv.close()
    assert st == [0] * 6
    for c, s, o in zip(csrs, srcs, outs):
        assert np.array_equal(mlmq.to_numpy(o), oracle.dijkstra(c, s)), s


def test_latency_probe_runs_and_leaves_graph_intact():
    """The latency probes (dependent relaxation hops, hand-off between two
    workgroups) return plausible times, and a solve afterwards is exact (the
    probe writes only its own scratch labels)."""
    mlmq = _mlmq()
    csr = gg.grid(200, 200, 0.05, seed=91)
    g = mlmq.Graph.from_csr(csr)
    hop_ns, hand_ns = mlmq.latency_probe(g, 100 * 200 + 100, 4096)
    _say(f"[probe] hop {hop_ns:.0f} ns, hand-off {hand_ns:.0f} ns")
    assert 10.0 < hop_ns < 1e5 and 10.0 < hand_ns < 1e5
    out = mlmq.sssp(g, 5)
    torch.cuda.synchronize()
    assert np.array_equal(mlmq.to_numpy(out), oracle.dijkstra(csr, 5))
    with pytest.raises(mlmq.MlmqError):
        mlmq.latency_probe(g, csr.n, 16)
    g.close()


def test_degree_ordered_copy_gathers_back():
    """Plain solves on a graph's degree-ordered copy (made by default for large
    power-law graphs, forced here with MLMQ_GRAPH_DEGREE_ORDER) are gathered
    back into the caller's vertex order: shortest paths into device and host
    buffers, and breadth-first levels, equal the oracle's, and so do those of
    the same graph created with MLMQ_GRAPH_KEEP_ORDER (no copy). RMAT-23 at
    full size, which gets the copy by default, is in the full-size tests."""
    mlmq = _mlmq()
    csr = gg.rmat(14, 16, seed=21)
    graphs = {"ordered": mlmq.Graph.from_csr(csr, degree_order=True),
              "kept": mlmq.Graph.from_csr(csr, keep_order=True)}
    with pytest.raises(mlmq.MlmqError):
        mlmq.Graph.from_csr(csr, keep_order=True, degree_order=True)
    srcs = [gg.max_degree_vertex(csr)] + [int(x) for x in gg.sample_sources(csr, 3, seed=4)]
    for s in srcs:
        want, levels = oracle.dijkstra(csr, s), oracle.bfs(csr, s)
        for name, g in graphs.items():
            _say(f"[ordered] {name} source {s}")
            out = mlmq.sssp(g, s)
            torch.cuda.synchronize()
            assert np.array_equal(mlmq.to_numpy(out), want), (name, s)
            host = np.empty(csr.n, dtype=np.uint32)
            mlmq.sssp(g, s, out=host)
            assert np.array_equal(host, want), (name, s)
            lv = mlmq.bfs(g, s)
            torch.cuda.synchronize()
            assert np.array_equal(mlmq.to_numpy(lv), levels), (name, s)
    for g in graphs.values():
        g.close()
