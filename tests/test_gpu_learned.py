"""What the trained stop network gains over the search without it.

On the 10,000 x 128 workload the whole learned-stop pipeline runs on the GPU
with the library's kernels: traces of the plain BF16 + rerank search on
training queries, FP32 training (forward, backward, Adam), BF16 export, and a
threshold calibrated on held-out training queries for a top-10 loss of at most
0.5% against the plain search. On the test queries the stopped search must
then take fewer hops than the same search without the network, lose at most
the calibrated share of its top-10, and never take more hops on any query.
"""
import json
import sys
from pathlib import Path

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DATA = Path(__file__).resolve().parent.parent / "data"


def say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_learned_stop_saves_hops_at_bounded_loss():
    p = DATA / "cfg1.deg"
    if not p.exists():
        pytest.skip("data/cfg1.deg not built (python -m oracle.build_graph --cfg 1)")
    from paper_2307_10479_amd import api, stop
    from synth.io import load_graph
    api.lib()
    adj, metric, _ = load_graph(p)
    meta = json.loads((DATA / "cfg1.meta.json").read_text())
    base, q, train = synth.cfg1(n_train=20_000)
    seed = meta["medoid"]
    store = api.VectorStore(dev(base), "bf16", metric)
    G = api.DeviceGraph(dev(adj))
    k, eps, interval = 10, 0.15, 4
    tr, ho = dev(train[:16_000]), dev(train[16_000:])
    seeds = lambda n: torch.full((n, 1), seed, dtype=torch.int32, device="cuda")
    say("learned stop: traces")
    X, y = stop.collect_traces(store, G, tr, seeds(tr.shape[0]), k, [eps], interval=interval,
                               rows=256)
    assert X.shape[0] > 10_000 and 0.0 < float(y.mean()) < 1.0
    mean, inv_std = stop.standardise(X)
    params, hist = stop.train(stop.standardised(X, mean, inv_std), y.contiguous(), epochs=6,
                              batch=4096)
    assert hist[-1] < hist[0]
    tau, table = stop.calibrate(store, G, ho, seeds(ho.shape[0]), k, eps, params, mean, inv_std,
                                interval)
    say("learned stop: tau", tau, [(t, round(a, 4), round(h, 1)) for t, a, h in table])
    assert tau < 1.0  # some threshold keeps the loss within 0.5% on the held-out queries
    model = stop.build_model(params, mean, inv_std, tau, interval)
    Q = dev(q)
    plain = api.search(store, G, Q, seeds(q.shape[0]), k, eps)
    got = api.search(store, G, Q, seeds(q.shape[0]), k, eps, stop=model)
    torch.cuda.synchronize()
    hp = plain[2][:, 0].cpu().numpy()
    hb = got[2][:, 0].cpu().numpy()
    agree = stop.top10_agreement(got[0], plain[0])
    say("learned stop: hops %.1f -> %.1f, top-10 agreement %.4f" % (hp.mean(), hb.mean(), agree))
    assert (hb <= hp).all()
    assert hb.mean() < 0.97 * hp.mean()
    assert agree >= 0.99  # calibrated for 0.995 on held-out queries; test queries are fresh
