"""Serving form on the GPU: queries submitted while others run are admitted as
slots and memory free up, and each result equals the oracle's (and so the
plain solve's) bit for bit. No device-wide synchronisation happens while a
server is alive: its resident kernel would hold it."""
import sys
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


def _graphs():
    big = gg.grid(40, 40, 0.0, seed=8)
    big.w[:] = (2**32 - 10) // 100  # not overflow-safe: exercises the exact check
    return [gg.grid(64, 64, 0.05, seed=1), gg.rmat(12, 8, seed=3), gg.uniform(5000, 40000, wmax=65535, seed=4),
            gg.grid(96, 80, 0.1, seed=2), big]


@pytest.fixture(scope="module")
def setup():
    mlmq = _mlmq()
    csrs = _graphs()
    return mlmq, csrs, [mlmq.Graph.from_csr(c) for c in csrs]


@pytest.mark.parametrize("slots,budget_mb", [(64, 4096), (3, 4096), (8, 2)])
def test_served_equals_alone(setup, slots, budget_mb):
    mlmq, csrs, graphs = setup
    rng = np.random.default_rng(slots * 1000 + budget_mb)
    nq = 60
    picks = [(int(g), int(rng.integers(0, csrs[g].n))) for g in rng.integers(0, len(csrs), nq)]
    outs = [mlmq.new_dist(csrs[g].n) for g, _ in picks]
    torch.cuda.synchronize()
    _say(f"[server] slots={slots} budget={budget_mb}MB queries={nq}")
    srv = mlmq.Server(graphs, mem_budget_bytes=budget_mb << 20, max_slots=slots)
    try:
        tickets = []
        for i, ((g, s), o) in enumerate(zip(picks, outs)):
            tickets.append(srv.submit(g, s, o))
            if i % 7 == 3:
                time.sleep(0.002)  # arrivals spread over time, some while others run
        status = [srv.wait(t, 30000) for t in tickets]
        times = [srv.times(t) for t in tickets]
    finally:
        srv.close()
    _say(f"[server] done, statuses {sorted(set(status))}")
    assert status == [0] * nq
    for a, b in times:
        assert 0 < a <= b
    for i, ((g, s), o) in enumerate(zip(picks, outs)):
        got = mlmq.to_numpy(o)
        want = oracle.dijkstra(csrs[g], s)
        assert np.array_equal(got, want), (i, g, s)


def test_server_result_matches_plain_solve(setup):
    mlmq, csrs, graphs = setup
    plain = mlmq.to_numpy(mlmq.sssp(graphs[1], 5))
    torch.cuda.synchronize()
    out = mlmq.new_dist(csrs[1].n)
    srv = mlmq.Server(graphs, mem_budget_bytes=1 << 30, max_slots=4)
    try:
        t = srv.submit(1, 5, out)
        assert srv.wait(t, 30000) == 0
        assert srv.poll(t) == 0
    finally:
        srv.close()
    assert np.array_equal(mlmq.to_numpy(out), plain)


def test_server_overflow_and_bad_arguments(setup):
    mlmq, csrs, graphs = setup
    of = gg.from_edges(4, [0, 1, 2], [1, 2, 3], [2**31, 2**31 - 1, 5])
    gof = mlmq.Graph.from_csr(of)
    out = mlmq.new_dist(4)
    out2 = mlmq.new_dist(csrs[0].n)
    torch.cuda.synchronize()
    srv = mlmq.Server([gof, graphs[0]], mem_budget_bytes=1 << 28, max_slots=2)
    try:
        t = srv.submit(0, 0, out)
        assert srv.wait(t, 30000) == mlmq.ERR_DISTANCE_OVERFLOW
        with pytest.raises(mlmq.MlmqError) as ei:
            srv.submit(2, 0, out)
        assert ei.value.code == mlmq.ERR_INVALID_ARG
        with pytest.raises(mlmq.MlmqError) as ei:
            srv.submit(1, csrs[0].n, out2)
        assert ei.value.code == mlmq.ERR_INVALID_ARG
        t2 = srv.submit(1, 0, out2)
        assert srv.wait(t2, 30000) == 0
    finally:
        srv.close()
    assert np.array_equal(mlmq.to_numpy(out2), oracle.dijkstra(csrs[0], 0))


def test_server_idle_relaunch(setup):
    """Resident waves leave after a stretch without work; a later query brings
    the kernel back."""
    mlmq, csrs, graphs = setup
    out = mlmq.new_dist(csrs[3].n)
    torch.cuda.synchronize()
    srv = mlmq.Server(graphs, mem_budget_bytes=1 << 28, max_slots=2)
    try:
        t = srv.submit(3, 1, out)
        assert srv.wait(t, 30000) == 0
        time.sleep(0.5)  # longer than the idle exit
        t = srv.submit(3, 2, out)
        assert srv.wait(t, 30000) == 0
    finally:
        srv.close()
    assert np.array_equal(mlmq.to_numpy(out), oracle.dijkstra(csrs[3], 2))
