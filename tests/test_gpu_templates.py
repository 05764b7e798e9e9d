"""Every candidate configuration the selector and the autotuner choose from
(and the feature-driven default) solves small graphs of each class to the
oracle's vector, element by element (integer arithmetic, tolerance 0); the
selector's pick and a tuned config do too."""
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


GRAPHS = {
    "road96x80": lambda: (gg.grid(96, 80, 0.1, seed=71), 40 * 80 + 17),
    "rmat13": lambda: (gg.rmat(13, 8, seed=72), None),
    "uniform4k-wide": lambda: (gg.uniform(4096, 30000, wmax=65535, seed=73), 5),
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_every_template_matches_oracle(name):
    mlmq = _mlmq()
    csr, src = GRAPHS[name]()
    if src is None:
        src = gg.max_degree_vertex(csr)
    want = oracle.dijkstra(csr, src)
    g = mlmq.Graph.from_csr(csr)
    out = mlmq.new_dist(csr.n)
    for t in range(-1, mlmq.candidate_count()):
        cfg = mlmq.candidate_config(g, t)
        _say(f"[templates] {name} t={t} {cfg.as_dict()}")
        out.fill_(7)
        mlmq.sssp(g, src, out=out, config=cfg)
        torch.cuda.synchronize()
        got = mlmq.to_numpy(out)
        assert np.array_equal(got, want), (name, t)
    sel = mlmq.select(g)
    mlmq.sssp(g, src, out=out, config=sel)
    torch.cuda.synchronize()
    assert np.array_equal(mlmq.to_numpy(out), want)
    tuned = mlmq.autotune(g, 300)
    mlmq.sssp(g, src, out=out)  # the tuned config is cached for cfg == NULL
    torch.cuda.synchronize()
    assert np.array_equal(mlmq.to_numpy(out), want), tuned.as_dict()
    g.close()
