"""Full-size workloads besides the headline one, each in one persistent launch in
the library's default configuration, with sampled queries checked one by one
against the oracle:

* 1,183,514 x 100 unit vectors (Zipf cluster sizes), inner product, exploratory
  search (each query is a base vertex, seeded at itself and excluded from its
  answer), k = 100, eps in {0, 0.1};
* 95,000 x 1,369 sparse lognormal vectors, L2, k = 100: FP32 traversal
  (bit-exact), BF16 and FP8-E4M3 (per-row scale) traversal each followed by the
  exact FP32 rerank of the pool (the oracle runs Algorithm 1 on the decoded
  vectors, then its own rerank), with recall@100 and the distance error against
  the FP64 ground truth reported for every precision;
* 2,000,000 x 300 anisotropic mixture, L2, degree 40: a stream of 100,000
  descriptors (k in {1, 10, 100}, eps in {0, 0.1, 0.2}, half exploratory) in
  one persistent launch.
"""
import json
import sys
from pathlib import Path

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DATA = Path(__file__).resolve().parent.parent / "data"


def say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def A():
    from paper_2307_10479_amd import api
    api.lib()
    return api


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _need(cfg, need_gt=True):
    p = DATA / ("cfg%d.deg" % cfg)
    gp = DATA / ("cfg%d.gt.npz" % cfg)
    if not p.exists() or not (DATA / ("cfg%d.meta.json" % cfg)).exists() or (need_gt and not gp.exists()):
        pytest.skip("data/cfg%d not built (python -m oracle.build_graph --cfg %d)" % (cfg, cfg))
    from synth.io import load_graph
    adj, metric, _ = load_graph(p)
    meta = json.loads((DATA / ("cfg%d.meta.json" % cfg)).read_text())
    gt = np.load(gp) if need_gt else None
    return adj, metric, meta, gt


def _parity(ids, ds, st, ref, what):
    rids, rds, rst = ref
    bad = np.nonzero((ids != rids).any(1) | (st[:, 0] != rst[:, 0]) | (st[:, 1] != rst[:, 1]))[0]
    assert len(bad) == 0, "%s: %d queries differ, first %d: gpu %s / oracle %s" % (
        what, len(bad), bad[0], st[bad[0]].tolist(), rst[bad[0]].tolist())
    fin = np.isfinite(rds)
    assert (np.isfinite(ds) == fin).all()
    assert (ds[fin] == rds[fin].astype(np.float32)).all(), what


def _recall(ids, gt_ids, k):
    hit = 0
    for a, b in zip(ids[:, :k], gt_ids[:, :k]):
        hit += len(set(a.tolist()) & set(b.tolist()))
    return hit / (k * len(ids))


def test_exploration_ip_full_size_sampled(A):
    adj, metric, meta, gt = _need(3)
    assert metric == oracle.IP
    base, qids = synth.cfg3()
    assert (gt["qids"] == qids).all()
    say("cfg3 full size")
    store = A.VectorStore(dev(base), "f32", metric)
    G = A.DeviceGraph(dev(adj))
    k = 100
    L = 16384  # the library's default capacity of S, passed explicitly
    sample = synth.rng(80).choice(len(qids), size=120, replace=False)
    rec = {}
    for eps in (0.0, 0.1):
        ids, ds, st = A.search_indexed(store, G, dev(qids), k, eps, queue_cap=L)
        torch.cuda.synchronize()
        ids, ds, st = ids.cpu().numpy(), ds.cpu().numpy(), st.cpu().numpy()
        assert not (ids == qids[:, None]).any()  # the query vertex is never returned
        ref = oracle.range_search_indexed(base, adj, qids[sample], k, eps, metric, cap_L=L,
                                          nthreads=oracle.nthreads_default())
        _parity(ids[sample], ds[sample], st[sample], ref, "cfg3 eps=%g" % eps)
        rec[eps] = _recall(ids, gt["ids"], k)
        say("cfg3 eps %.1f recall@100 %.4f hops %.1f" % (eps, rec[eps], st[:, 0].mean()))
    assert rec[0.1] >= rec[0.0]


def test_precision_stress_full_size(A):
    adj, metric, meta, gt = _need(4)
    base, q = synth.cfg4()
    n, m = base.shape
    seed = meta["medoid"]  # float data: both sides start from the oracle's FP64 medoid
    say("cfg4 full size")
    G = A.DeviceGraph(dev(adj))
    xb = dev(base)
    k, eps = 100, 0.1
    L = 16384  # the library's default capacity of S, passed explicitly
    seeds = dev(np.full((q.shape[0], 1), seed, np.int32))
    sample = synth.rng(81).choice(q.shape[0], size=60, replace=False)
    nthr = oracle.nthreads_default()
    table = {}
    for dtype in ("f32", "bf16", "fp8"):
        store = A.VectorStore(xb, dtype, metric)
        ids, ds, st = A.search(store, G, dev(q), seeds, k, eps, queue_cap=L)
        torch.cuda.synchronize()
        ids, ds, st = ids.cpu().numpy(), ds.cpu().numpy(), st.cpu().numpy()
        if dtype == "f32":
            ref = oracle.range_search(base, adj, q[sample], [seed], k, eps, metric, cap_L=L,
                                      nthreads=nthr)
            _parity(ids[sample], ds[sample], st[sample], ref, "cfg4 f32")
        else:
            if dtype == "bf16":
                xd = oracle.bf16_decode(oracle.bf16_encode(base))
            else:
                codes, scale = oracle.fp8_encode_rows(base)
                xd = oracle.fp8_decode_rows(codes, scale, m)
            pids, pds, pst = oracle.range_search(xd, adj, q[sample], [seed], k, eps, metric,
                                                 cap_L=L, nthreads=nthr)
            assert (st[sample, 0] == pst[:, 0]).all() and (st[sample, 1] == pst[:, 1]).all(), dtype
            for j, i in enumerate(sample):
                rid, rd = oracle.rerank(base, q[i], pids[j], k, metric)
                assert ids[i].tolist() == rid.tolist(), (dtype, i)
                assert (ds[i] == rd).all(), (dtype, i)
        # against the FP64 ground truth: ranking (recall) and distance rounding
        d64 = np.array([[oracle.dist64(base[j], q[i]) for j in ids[i][:10]] for i in sample])
        rel = np.abs(ds[sample][:, :10].astype(np.float64) - d64) / np.maximum(d64, 1e-30)
        table[dtype] = dict(recall=_recall(ids, gt["ids"], k), max_rel_err=float(rel.max()),
                            hops=float(st[:, 0].mean()), evals=float(st[:, 1].mean()))
        say("cfg4", dtype, table[dtype])
        # every returned distance is an FP32 sum of m non-negative terms: within
        # (m - 1) unit roundoffs of the exact value
        assert rel.max() <= (m - 1) * 2.0 ** -24
    assert table["bf16"]["recall"] >= table["f32"]["recall"] - 0.05
    assert table["fp8"]["recall"] >= table["f32"]["recall"] - 0.10


def test_batch_stream_full_size_sampled(A):
    adj, metric, meta, _ = _need(5, need_gt=False)
    base, q, desc = synth.cfg5()
    seed = meta["medoid"]
    nq = q.shape[0]
    kind = desc["indexed"]
    sv = np.where(kind == 1, desc["vertex"], seed).astype(np.int32)
    kk, ee = desc["k"], desc["eps"]
    descs, total, kmax = A.make_descs(kind, sv, np.arange(nq, dtype=np.int64), kk, ee)
    L = 16384  # the library's default capacity of S, passed explicitly
    say("cfg5 batch", nq, total, kmax)
    store = A.VectorStore(dev(base), "f32", metric)
    G = A.DeviceGraph(dev(adj))
    ids, ds, st = A.search_batch(store, G, dev(q), descs, nq, total, kmax, queue_cap=L)
    torch.cuda.synchronize()
    ids, ds, st = ids.cpu().numpy(), ds.cpu().numpy(), st.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(kk)[:-1]])
    sample = synth.rng(82).choice(nq, size=150, replace=False)
    for i in sample:
        if kind[i] == 1:
            rid, rd, rst = oracle.range_search_indexed(base, adj, [sv[i]], int(kk[i]), float(ee[i]),
                                                       metric, cap_L=L)
        else:
            rid, rd, rst = oracle.range_search(base, adj, q[i:i + 1], [seed], int(kk[i]),
                                               float(ee[i]), metric, cap_L=L)
        sl = slice(off[i], off[i] + kk[i])
        assert ids[sl].tolist() == rid[0].tolist(), i
        assert (ds[sl] == rd[0].astype(np.float32)).all(), i
        assert st[i, 0] == rst[0, 0] and st[i, 1] == rst[0, 1], i
    say("cfg5 hops mean %.1f, evals mean %.1f" % (st[:, 0].mean(), st[:, 1].mean()))
