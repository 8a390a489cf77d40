"""Host-side logic of the package: recall (Eq. recall@k)."""
import numpy as np
import pytest


def test_recall_definition():
    from paper_2307_10479_amd import metrics
    gt = np.array([[1, 2, 3, 4], [5, 6, 7, 8]])
    got = np.array([[4, 3, 9, 9], [5, 6, 7, 8]])
    assert metrics.recall_at_k(got, gt, 4) == pytest.approx((2 / 4 + 1) / 2)
    assert metrics.recall_at_k(got, gt, 2) == pytest.approx((0 + 1) / 2)




def test_graph_file_round_trip(tmp_path):
    """Both graph file versions give back the graph: version 1 byte for byte,
    version 2 with every row's neighbours in ascending order and the weights
    permuted alongside."""
    import numpy as np

    import synth
    from synth.io import load_graph, save_graph
    r = synth.rng(5)
    n, d = 5000, 30
    adj = np.stack([r.choice(n, size=d, replace=False) for _ in range(n)]).astype(np.int32)
    w = r.random((n, d)).astype(np.float32)
    p1, p2 = tmp_path / "a.deg", tmp_path / "b.deg"
    save_graph(p1, adj, 1, w, compact=False)
    save_graph(p2, adj, 1, w)
    a1, m1, w1 = load_graph(p1, with_weights=True)
    a2, m2, w2 = load_graph(p2, with_weights=True)
    assert m1 == m2 == 1
    assert (a1 == adj).all() and (w1 == w).all()
    order = np.argsort(adj, axis=1)
    assert (a2 == np.take_along_axis(adj, order, axis=1)).all()
    assert (w2 == np.take_along_axis(w, order, axis=1)).all()
    assert p2.stat().st_size < p1.stat().st_size
