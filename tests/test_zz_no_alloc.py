"""The allocation-free entry point (mlmq_sssp_noalloc) through the C ABI: its
output equals mlmq_sssp's (and the oracle's) bit for bit, on two calls in a
row, the second on a smaller input, and sizes beyond its fixed array are
refused with a clear error."""
import sys

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


def _cases():
    big = gg.grid(300, 300, 0.05, seed=31)
    small = gg.rmat(12, 8, seed=32)
    return [("grid300", big, 150 * 300 + 150), ("rmat12", small, gg.max_degree_vertex(small))]


def test_noalloc_matches_sssp_twice_shrinking():
    mlmq = _mlmq()
    for rep in range(2):
        for name, csr, src in _cases():
            g = mlmq.Graph.from_csr(csr)
            _say(f"[noalloc] rep={rep} {name} n={csr.n} m={csr.m} src={src}")
            ref = mlmq.new_dist(csr.n)
            mlmq.sssp(g, src, out=ref)
            out = mlmq.new_dist(csr.n)
            out.fill_(7)
            _, st = mlmq.sssp_noalloc(g, src, out, stats=True)
            torch.cuda.synchronize()
            got = mlmq.to_numpy(out)
            assert np.array_equal(got, mlmq.to_numpy(ref)), name
            assert np.array_equal(got, oracle.dijkstra(csr, src)), name
            assert st["status"] == 0 and st["expansions"] >= int((got != oracle.UNREACHABLE).sum())
            g.close()


def test_noalloc_queue_configs_and_overflow_check():
    """Bucket L2 and near-far L1 through the fixed array, and the exact
    overflow test (a saturating candidate that is not a shortest path)."""
    mlmq = _mlmq()
    csr = gg.grid(96, 80, 0.1, seed=2)
    g = mlmq.Graph.from_csr(csr)
    src = 40 * 80 + 33
    want = oracle.dijkstra(csr, src)
    for kw in (dict(l0_rows=1, l1_type=2, l2_type=1, bmax=32, bnum=2, delta2_log2=5, delta1=32, th_hub=0),
               dict(l0_rows=2, l1_type=1, l2_type=0, th_hub=0)):
        out = mlmq.new_dist(csr.n)
        mlmq.sssp_noalloc(g, src, out, config=mlmq.default_config(**kw))
        torch.cuda.synchronize()
        assert np.array_equal(mlmq.to_numpy(out), want), kw
    g.close()
    fa = gg.from_edges(3, [0, 1, 0], [1, 2, 2], [2**31, 2**31, 5])
    g = mlmq.Graph.from_csr(fa)
    out = mlmq.new_dist(3)
    mlmq.sssp_noalloc(g, 0, out)
    torch.cuda.synchronize()
    assert mlmq.to_numpy(out).tolist() == [0, 2**31, 5]
    g.close()


def test_noalloc_refuses_oversized_plan_and_host_output():
    mlmq = _mlmq()
    csr = gg.grid(64, 64, 0.0, seed=1)
    g = mlmq.Graph.from_csr(csr)
    out = mlmq.new_dist(csr.n)
    with pytest.raises(mlmq.MlmqError) as ei:
        mlmq.sssp_noalloc(g, 0, out, config=mlmq.default_config(l2_capacity=1 << 25))
    assert ei.value.code == mlmq.ERR_INVALID_ARG and "exceeds" in str(ei.value)
    host = np.empty(csr.n, np.uint32)
    rc = mlmq.lib().mlmq_sssp_noalloc(g.handle, 0, host.ctypes.data, None)
    assert rc == mlmq.ERR_INVALID_ARG
    # the entry point still works after the refusals
    mlmq.sssp_noalloc(g, 0, out)
    torch.cuda.synchronize()
    assert np.array_equal(mlmq.to_numpy(out), oracle.dijkstra(csr, 0))
    g.close()
