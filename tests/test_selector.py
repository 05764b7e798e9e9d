"""The learned configuration selector (Section 3.5) on the host: its model
inputs, the C tables against the training library's own predictions, and its
quality on the held-out graphs of the timing corpus (graphs the forest never
saw), compared with the best fixed template and the feature-driven default,
in the paper's terms: the share of graphs whose pick runs within 0.9 of the
best template's speed, and whether the best template is among the top three."""
import json
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SEL = os.path.join(ROOT, "paper_2602_10080_amd", "selector")


def _mlmq():
    import paper_2602_10080_amd as mlmq
    return mlmq


def _train():
    from paper_2602_10080_amd.selector import train
    return train


def test_template_inputs():
    mlmq = _mlmq()
    k = mlmq.candidate_count()
    assert k >= 40
    f = dict(n=1 << 20, nnz=16 << 20, avg_deg=16.0, max_deg=5000.0, std_deg=40.0, avg_w=128.0, std_w=73.0,
             max_w=255.0)
    xs = np.array([mlmq.select_inputs(f, t) for t in range(k)])
    assert xs.shape == (k, 20)
    # graph part identical for every template, knob part distinct
    assert np.all(xs[:, :8] == xs[0, :8])
    assert xs[0, 0] == pytest.approx(20.0) and xs[0, 1] == pytest.approx(24.0)
    assert xs[0, 4] == pytest.approx(40.0 / 16.0) and xs[0, 5] == pytest.approx(7.0)
    assert len({tuple(r) for r in xs[:, 8:]}) == k
    with pytest.raises(mlmq.MlmqError):
        mlmq.select_inputs(f, k)
    order, scores = mlmq.select_rank(f)
    assert sorted(order.tolist()) == list(range(k))
    assert np.all(np.diff(scores[order]) <= 0)


def test_c_tables_reproduce_training_predictions():
    mlmq = _mlmq()
    cases = json.load(open(os.path.join(SEL, "model_check.json")))["cases"]
    assert len(cases) >= 100
    worst = 0.0
    for c in cases:
        _, scores = mlmq.select_rank(c["features"])
        worst = max(worst, abs(float(scores[c["template"]]) - c["prediction"]))
    assert worst < 1e-6


def test_heldout_quality():
    mlmq = _mlmq()
    train = _train()
    k = mlmq.candidate_count()
    graphs = train.load_corpus(os.path.join(SEL, "corpus.csv"))
    test = {gi: g for gi, g in graphs.items() if g["split"] == "test"}
    assert len(test) >= 20 and len(graphs) - len(test) >= 50
    rows = train.evaluate(graphs, k, lambda g: mlmq.select_rank(g["features"])[0].tolist())
    train_r = np.array([train.relative(g, k)[0] for g in graphs.values() if g["split"] == "train"])
    fixed = int(np.argmax(train_r.mean(axis=0)))
    rows_fixed = train.evaluate(graphs, k, lambda g: [fixed] + [t for t in range(k) if t != fixed])
    sel09 = np.mean([r["top1"] >= 0.9 for r in rows])
    top3 = np.mean([r["best_in_top3"] for r in rows])
    top3_09 = np.mean([r["top3_best"] >= 0.9 for r in rows])
    fix09 = np.mean([r["top1"] >= 0.9 for r in rows_fixed])
    print(f"held-out: selector within 0.9 {sel09:.2f}, best in top 3 {top3:.2f}, top-3 within 0.9 "
          f"{top3_09:.2f}; best fixed template {fixed} within 0.9 {fix09:.2f}")
    # measured on this corpus: selector 0.96 within 0.9 (best fixed template 0.73), best template among
    # the top three on 22 of 26 held-out graphs (several templates often lie within a few percent of each
    # other there), one of the top three within 0.9 on 25 of 26
    assert sel09 >= fix09 + 0.15 and sel09 >= 0.85
    assert np.mean([r["top1"] for r in rows]) >= np.mean([r["top1"] for r in rows_fixed])
    assert top3 >= 0.8
    assert top3_09 >= 0.9
