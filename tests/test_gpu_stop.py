"""GPU parity of the learned-stop path and of the visited set's growth.

The trace rows (16 features, label) of the HIP search are compared element
by element with the oracle's, and a search stopped by a BF16 network trained
with the library's kernels returns the oracle's ids, distances, hops,
evaluations and stop flags (BF16 inference is one fixed FP32 computation on
both sides, so every stop decision is the same). The visited set must stay
exact when a query checks far more vertices than the first workspace table
holds, including the shared tables sized for all n vertices."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def A():
    from paper_2307_10479_amd import api
    api.lib()
    return api


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


_G = {}


def graph(n=1500, m=24, d=16, seed=3):
    key = (n, m, d, seed)
    if key not in _G:
        x = synth.small_int(seed, n, m, hi=64)
        adj, _, _ = oracle.build_graph(x, d, k_ext=2 * d, eps_ext=0.2, k_opt=d)
        _G[key] = (x, adj)
    return _G[key]


def gpu_trace(A, x, adj, q, k, eps, rows, itv, L, indexed=False, **kw):
    store = A.VectorStore(dev(x), "f32")
    g = A.DeviceGraph(dev(adj))
    nq = q.shape[0]
    tr = torch.full((nq * rows * A.TRACE_W,), -5.0, dtype=torch.float32, device="cuda")
    if indexed:
        ids, ds, st = A.search_indexed(store, g, dev(q), k, eps, queue_cap=L, trace=tr,
                                       trace_rows=rows, trace_interval=itv, **kw)
    else:
        ids, ds, st = A.search(store, g, dev(q), dev(np.zeros((nq, 1), np.int32)), k, eps,
                               queue_cap=L, trace=tr, trace_rows=rows, trace_interval=itv, **kw)
    torch.cuda.synchronize()
    return (ids.cpu().numpy(), ds.cpu().numpy(), st.cpu().numpy(),
            tr.view(nq, rows, A.TRACE_W).cpu().numpy())


def assert_trace_equal(got, ref, what):
    lab = ref[:, :, 16]
    assert (got[:, :, 16] == lab).all(), what + ": labels differ"
    w = lab >= 0
    g, r = got[:, :, :16][w], ref[:, :, :16][w]
    bad = g != r
    if bad.any():
        cols = np.nonzero(bad.any(0))[0]
        i = np.nonzero(bad.any(1))[0][0]
        raise AssertionError("%s: features differ in columns %s (rows per column %s); first row "
                             "gpu %s oracle %s" % (what, cols.tolist(), bad.sum(0)[cols].tolist(),
                                                   g[i].tolist(), r[i].tolist()))
    assert (got[:, :, 17:19][w] == ref[:, :, 17:19][w]).all(), what + ": query/hop columns differ"


@pytest.mark.parametrize("k,eps,itv,L", [(10, 0.0, 1, 4096), (10, 0.1, 4, 4096), (1, 0.2, 3, 4096),
                                         (50, 0.1, 8, 4096), (10, 0.2, 2, 16)])
def test_trace_rows_equal_the_oracle(A, k, eps, itv, L):
    x, adj = graph()
    q = synth.small_int(30, 200, 24, hi=64)
    say("trace rows", k, eps, itv, L)
    ids, ds, st, tr = gpu_trace(A, x, adj, q, k, eps, 96, itv, L)
    rids, rds, rst, rtr = oracle.range_search(x, adj, q, [0], k, eps, cap_L=L, trace_rows=96,
                                              trace_interval=itv)
    assert (ids == rids).all() and (st[:, 0] == rst[:, 0]).all() and (st[:, 1] == rst[:, 1]).all()
    assert ((st[:, 2] & A.FLAG_QUEUE_OVERFLOW != 0) == (rst[:, 3] & 1 != 0)).all()
    assert_trace_equal(tr, rtr, "trace k=%d eps=%g" % (k, eps))


def test_trace_rows_exploratory_equal_the_oracle(A):
    x, adj = graph()
    qids = np.arange(0, 1500, 7, dtype=np.int32)
    say("trace rows exploratory")
    ids, ds, st, tr = gpu_trace(A, x, adj, qids, 10, 0.1, 64, 2, 4096, indexed=True)
    rids, rds, rst, rtr = oracle.range_search_indexed(x, adj, qids, 10, 0.1, cap_L=4096,
                                                      trace_rows=64, trace_interval=2)
    assert (ids == rids).all() and (st[:, 0] == rst[:, 0]).all()
    assert_trace_equal(tr, rtr, "trace exploratory")


def _trained_model(A, X, y, seed=0):
    from paper_2307_10479_amd import stop
    Xt, yt = dev(X), dev(y)
    mean, inv_std = stop.standardise(Xt)
    params, hist = stop.train(stop.standardised(Xt, mean, inv_std), yt.contiguous(), epochs=3,
                              batch=1024, seed=seed)
    w = A.mlp_export_bf16(params)
    torch.cuda.synchronize()
    return w, mean, inv_std, hist


@pytest.mark.parametrize("quant,itv,L", [(0.6, 4, 4096), (0.9, 2, 4096), (0.75, 3, 24)])
def test_stopped_search_with_a_trained_network_equals_the_oracle(A, quant, itv, L):
    x, adj = graph()
    tq = synth.small_int(31, 1500, 24, hi=64)
    say("stop: traces", quant, itv)
    _, _, _, tr = oracle.range_search(x, adj, tq, [0], 10, 0.1, cap_L=L, trace_rows=64,
                                      trace_interval=itv)
    rows = tr.reshape(-1, 20)
    rows = rows[rows[:, 16] >= 0]
    w, mean, inv_std, hist = _trained_model(A, rows[:, :16].copy(), rows[:, 16].copy())
    assert hist[-1] < hist[0]
    from paper_2307_10479_amd import stop
    # tau: the network's probability at the `quant` quantile of the training rows,
    # so that a share of the queries stop early and the others run to the end
    fs = stop.standardised(dev(rows[:, :16].copy()), mean, inv_std).cpu().numpy()
    z = oracle.mlp_logits_bf16(w.cpu().numpy(), fs)
    tau = float(1.0 / (1.0 + np.exp(-np.quantile(z, quant))))
    model = stop.build_model_from_bf16(w, mean, inv_std, tau, itv)
    q = synth.small_int(32, 300, 24, hi=64)
    store = A.VectorStore(dev(x), "f32")
    g = A.DeviceGraph(dev(adj))
    ids, ds, st = A.search(store, g, dev(q), dev(np.zeros((300, 1), np.int32)), 10, 0.1,
                           queue_cap=L, stop=model)
    torch.cuda.synchronize()
    om = oracle.StopModel(w.cpu().numpy(), mean.cpu().numpy(), inv_std.cpu().numpy(), tau, itv)
    rids, rds, rst = oracle.range_search(x, adj, q, [0], 10, 0.1, cap_L=L, stop=om)
    ids, ds, st = ids.cpu().numpy(), ds.cpu().numpy(), st.cpu().numpy()
    stopped = (rst[:, 3] & 16) != 0
    say("stop: oracle stops %d of 300" % stopped.sum())
    assert 0 < stopped.sum() < 300
    assert (ids == rids).all() and (ds == rds).all()
    assert (st[:, 0] == rst[:, 0]).all() and (st[:, 1] == rst[:, 1]).all()
    assert ((st[:, 2] & A.FLAG_LEARNED_STOP != 0) == stopped).all()


def test_batch_trace_rows_and_skipped_descriptor_labels(A):
    x, adj = graph()
    nq = 60
    r = synth.rng(33)
    q = synth.small_int(34, nq, 24, hi=64)
    kind = (r.random(nq) < 0.5).astype(np.int32)
    kk = r.choice(np.array([1, 10, 40], np.int32), size=nq)
    ee = r.choice(np.array([0.0, 0.1, 0.2], np.float32), size=nq)
    vert = r.integers(0, 1500, size=nq).astype(np.int32)
    sv = np.where(kind == 1, vert, 0).astype(np.int32)
    rows = np.arange(nq, dtype=np.int64)
    rows[7] = 10_000  # outside the query rows: skipped
    descs, total, kmax = A.make_descs(kind, sv, rows, kk, ee)
    store = A.VectorStore(dev(x), "f32")
    g = A.DeviceGraph(dev(adj))
    tr = torch.full((nq * 32 * A.TRACE_W,), 3.0, dtype=torch.float32, device="cuda")
    say("batch trace")
    ids, ds, st = A.search_batch(store, g, dev(q), descs, nq, total, kmax, queue_cap=4096,
                                 trace=tr, trace_rows=32, trace_interval=2)
    torch.cuda.synchronize()
    tr = tr.view(nq, 32, A.TRACE_W).cpu().numpy()
    assert (tr[7, :, 16] == -1).all()
    for i in range(nq):
        if i == 7:
            continue
        if kind[i] == 1:
            ref = oracle.range_search_indexed(x, adj, [vert[i]], int(kk[i]), float(ee[i]),
                                              cap_L=4096, trace_rows=32, trace_interval=2)
        else:
            ref = oracle.range_search(x, adj, q[i:i + 1], [0], int(kk[i]), float(ee[i]),
                                      cap_L=4096, trace_rows=32, trace_interval=2,
                                      kind=np.zeros(1, np.int32))
        rtr = ref[3].copy()
        rtr[:, :, 17] = i
        assert_trace_equal(tr[i:i + 1], rtr, "batch descriptor %d" % i)


# ---------------------------------------------------------------- visited set growth
def circulant(n, d):
    """The d-regular circulant graph (v joined to v +- 1..d/2 mod n): connected."""
    off = [o for j in range(1, d // 2 + 1) for o in (j, -j)]
    v = np.arange(n, dtype=np.int64)[:, None]
    return ((v + np.array(off)[None, :]) % n).astype(np.int32)


@pytest.mark.parametrize("n,nq", [(60_000, 16), (120_000, 150)])
def test_visited_set_exact_beyond_the_first_tables(A, n, nq):
    # eps = inf on a connected graph checks every vertex: 60k ids pass the
    # region's 8K and 32K tables into its 128K table; 120k ids need a shared
    # table (more queries than shared tables: some wait for one)
    x = synth.small_float(35, n, 4)
    adj = circulant(n, 8)
    q = synth.small_float(36, nq, 4)
    say("visited growth", n, nq)
    store = A.VectorStore(dev(x), "f32")
    g = A.DeviceGraph(dev(adj))
    ids, ds, st = A.search(store, g, dev(q), dev(np.zeros((nq, 1), np.int32)), 10, float("inf"),
                           queue_cap=1024, hash_slots=256)
    torch.cuda.synchronize()
    ids, ds, st = ids.cpu().numpy(), ds.cpu().numpy(), st.cpu().numpy()
    rids, rds, rst = oracle.range_search(x, adj, q, [0], 10, float("inf"), cap_L=1024)
    assert (rst[:, 1] == n).all() and (st[:, 1] == n).all()
    assert (ids == rids).all() and (ds == rds).all() and (st[:, 0] == rst[:, 0]).all()
    assert (st[:, 2] & A.FLAG_HASH_FULL == 0).all()
