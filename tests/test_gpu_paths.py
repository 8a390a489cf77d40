"""GPU tests of the other library paths against the oracle: the BF16/FP8
stores and the FP32 rerank, the medoid seed, brute-force ground truth on
matrix cores, the stop-predictor MLP kernels, the batched persistent launch
and the trace/learned-stop hooks."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BIG_L = 4096


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


def graph(n, m, d, kind="int", metric=oracle.L2, seed=0):
    key = (n, m, d, kind, metric, seed)
    if key not in _G:
        if kind == "int":
            x = synth.small_int(seed, n, m, hi=256)
        elif kind == "unit":
            x = synth.small_unit(seed, n, m)
        elif kind == "sparse":
            x = synth.small_float(seed, n, m)
            x = np.where(synth.rng(seed).random(x.shape) < 0.8, 0.0, np.exp(x)).astype(np.float32)
        else:
            x = synth.small_float(seed, n, m)
        adj, w, _ = oracle.build_graph(x, d, metric, k_ext=2 * d, eps_ext=0.2, k_opt=d)
        _G[key] = (x, adj)
    return _G[key]


# ---------------------------------------------------------------- encoders
def test_bf16_encoder_matches_oracle(A):
    x = synth.small_float(1, 300, 37) * 1000
    say("bf16 encoder")
    st = A.VectorStore(dev(x), "bf16")
    torch.cuda.synchronize()
    got = st.data.cpu().numpy()[:, :37]
    assert (got == oracle.bf16_encode(x)).all()
    assert (st.data.cpu().numpy()[:, 37:] == 0).all()


def test_fp8_encoder_matches_oracle(A):
    x = synth.small_float(2, 400, 101) * 7
    x[3] = 0.0
    x[5, :] = np.float32(1e-3)
    say("fp8 encoder")
    st = A.VectorStore(dev(x), "fp8")
    torch.cuda.synchronize()
    codes, scale = oracle.fp8_encode_rows(x)
    assert (st.scale.cpu().numpy() == scale).all()
    assert (st.data.cpu().numpy()[:, :101] == codes).all()


# ---------------------------------------------------------------- precision path
def test_bf16_lossless_on_integer_data(A):
    x, adj = graph(1500, 32, 30, "int")
    q = synth.small_int(3, 200, 32, hi=256)
    say("bf16 lossless")
    g = A.DeviceGraph(dev(adj))
    s32 = A.VectorStore(dev(x), "f32")
    s16 = A.VectorStore(dev(x), "bf16")
    seeds = dev(np.zeros((200, 1), np.int32))
    a = A.search(s32, g, dev(q), seeds, 10, 0.1, queue_cap=BIG_L)
    b = A.search(s16, g, dev(q), seeds, 10, 0.1, queue_cap=BIG_L)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert (u.cpu().numpy() == v.cpu().numpy()).all()
    ref = oracle.range_search(x, adj, q, [0], 10, 0.1, cap_L=BIG_L)
    assert (a[0].cpu().numpy() == ref[0]).all()


@pytest.mark.parametrize("dtype,kind,metric,m", [("bf16", "float", oracle.L2, 64),
                                                 ("bf16", "unit", oracle.IP, 100),
                                                 ("fp8", "sparse", oracle.L2, 137),
                                                 ("fp8", "float", oracle.L2, 300)])
@pytest.mark.parametrize("k,pool", [(10, 10), (10, 40), (100, 200), (300, 1000)])
def test_reduced_precision_with_rerank_matches_oracle(A, dtype, kind, metric, m, k, pool):
    """Traversal over decoded values then FP32 rerank of the pool: the oracle runs
    Algorithm 1 on the decoded vectors with k = pool, then reranks in FP32."""
    x, adj = graph(1200, m, 20, kind, metric)
    q = synth.small_float(4, 120, m) if kind != "unit" else synth.small_unit(4, 120, m)
    if kind == "sparse":
        q = np.abs(q)
    say("precision", dtype, kind, m, k, pool)
    store = A.VectorStore(dev(x), dtype, metric)
    g = A.DeviceGraph(dev(adj))
    ids, ds, st = A.search(store, g, dev(q), dev(np.zeros((120, 1), np.int32)), k, 0.1,
                           k_pool=pool, queue_cap=BIG_L)
    torch.cuda.synchronize()
    ids, ds, st = ids.cpu().numpy(), ds.cpu().numpy(), st.cpu().numpy()
    if dtype == "bf16":
        xd = oracle.bf16_decode(oracle.bf16_encode(x))
    else:
        codes, scale = oracle.fp8_encode_rows(x)
        xd = oracle.fp8_decode_rows(codes, scale, m)
    pids, pds, pst = oracle.range_search(xd, adj, q, [0], pool, 0.1, metric, cap_L=BIG_L)
    assert (st[:, 0] == pst[:, 0]).all() and (st[:, 1] == pst[:, 1]).all()
    for i in range(120):
        rid, rd = oracle.rerank(x, q[i], pids[i], k, metric)
        assert ids[i].tolist() == rid.tolist(), i
        assert (ds[i] == rd).all(), i


# ---------------------------------------------------------------- medoid
@pytest.mark.parametrize("kind,metric", [("int", oracle.L2), ("unit", oracle.IP)])
def test_medoid_matches_oracle(A, kind, metric):
    x = synth.small_int(5, 20000, 24, hi=256) if kind == "int" else synth.small_unit(5, 20000, 24)
    say("medoid", kind)
    got = A.medoid(dev(x), metric)
    ref = oracle.medoid(x, metric)
    if kind == "int":
        assert got == ref
    else:  # float sums in another order: the chosen vertex must be optimal to rounding
        mean = x.astype(np.float64).mean(0)
        s = x.astype(np.float64) @ mean
        assert s[got] >= s[ref] - 1e-12


# ---------------------------------------------------------------- brute force
# integer data of magnitude <= 255 with at most 128 dims takes the exact BF16 matrix-core
# path; 129..300 dims (and any non-integer value) the FP32 path: both must equal FP64
@pytest.mark.parametrize("n,nq,m,k", [(5000, 300, 128, 10), (7000, 130, 24, 100), (3000, 64, 37, 1),
                                      (9000, 200, 128, 1000), (4100, 257, 130, 1024),
                                      (6000, 140, 300, 64)])
def test_knn_integer_exact(A, n, nq, m, k):
    x = synth.small_int(6, n, m, hi=256)
    q = synth.small_int(7, nq, m, hi=256)
    say("knn int", n, nq, m, k)
    ids, ds = A.knn_bruteforce(dev(x), dev(q), k)
    torch.cuda.synchronize()
    rids, rds = oracle.knn64(x, q, k)
    assert (ids.cpu().numpy() == rids).all()
    assert (ds.cpu().numpy().astype(np.float64) == rds).all()


@pytest.mark.parametrize("kind,metric,m", [("float", oracle.L2, 100), ("unit", oracle.IP, 100),
                                           ("sparse", oracle.L2, 300)])
def test_knn_float_tolerance(A, kind, metric, m):
    x, _ = (synth.small_float(8, 6000, m), None)
    if kind == "unit":
        x = synth.small_unit(8, 6000, m)
    if kind == "sparse":
        x = np.where(synth.rng(8).random(x.shape) < 0.8, 0.0, np.exp(x)).astype(np.float32)
    q = x[:200] + 0.01 * synth.small_float(9, 200, m)
    if kind == "unit":
        q = q / np.linalg.norm(q, axis=1, keepdims=True)
    q = q.astype(np.float32)
    say("knn float", kind)
    ids, ds = A.knn_bruteforce(dev(x), dev(q), 20, metric)
    torch.cuda.synchronize()
    ids, ds = ids.cpu().numpy(), ds.cpu().numpy()
    rids, rds = oracle.knn64(x, q, 20, metric)
    for i in range(200):
        if ids[i].tolist() != rids[i].tolist():
            # only swaps between entries whose FP64 distances differ by <= 1e-6 relative
            assert set(ids[i]) ^ set(rids[i]) <= set(
                j for j in range(6000) if abs(oracle.dist64(x[j], q[i], metric) - rds[i, -1]) <=
                1e-6 * max(1.0, abs(rds[i, -1]))), i
        assert np.allclose(ds[i], rds[i], rtol=1e-6, atol=1e-6)


def test_knn_fp32_path_on_half_integer_queries(A):
    # one non-integer query value sends every query to the FP32 path; values are
    # multiples of 1/2 below 128, so FP32 products and sums are still exact
    x = synth.small_int(11, 5000, 64, hi=128).astype(np.float32)
    q = synth.small_int(12, 150, 64, hi=128).astype(np.float32)
    q[3, 5] += 0.5
    say("knn fp32 path")
    ids, ds = A.knn_bruteforce(dev(x), dev(q), 50)
    torch.cuda.synchronize()
    rids, rds = oracle.knn64(x, q, 50)
    assert (ids.cpu().numpy() == rids).all()
    assert (ds.cpu().numpy().astype(np.float64) == rds).all()


def test_knn_exclude(A):
    x = synth.small_int(10, 4000, 16, hi=256)
    qids = np.arange(0, 4000, 37, dtype=np.int32)
    say("knn exclude")
    ids, ds = A.knn_bruteforce(dev(x), dev(x[qids]), 10, exclude=dev(qids))
    torch.cuda.synchronize()
    rids, rds = oracle.knn64(x, x[qids], 10, exclude=qids)
    assert (ids.cpu().numpy() == rids).all()


# ---------------------------------------------------------------- MLP
def _mlp_data(B, seed):
    X = synth.small_float(seed, B, 16)
    y = (synth.rng(seed).random(B) < 0.4).astype(np.float32)
    P = synth.rng(seed + 1).standard_normal(5313) * 0.2
    return P, X, y


@pytest.mark.parametrize("B", [1, 31, 32, 1000, 4099])
def test_mlp_forward_backward_vs_oracle(A, B):
    P, X, y = _mlp_data(B, 11)
    say("mlp", B)
    Pt = dev(P.astype(np.float32))
    grad = torch.empty(5313, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    A.mlp_train_step(Pt, None, None, dev(X), dev(y), 1, 0.0, grad=grad, loss=loss)
    logits = A.mlp_forward(Pt, dev(X))
    torch.cuda.synchronize()
    rl, rg, rz = oracle.mlp_fwd_bwd(P.astype(np.float32).astype(np.float64), X, y)
    assert abs(loss.item() - rl) <= 1e-5 * max(1.0, abs(rl))
    g = grad.cpu().numpy().astype(np.float64)
    scale = np.abs(rg).max()
    assert np.abs(g - rg).max() <= 1e-4 * scale
    assert np.allclose(logits.cpu().numpy(), rz, rtol=1e-4, atol=1e-4)


def test_mlp_adam_step_vs_oracle(A):
    P, X, y = _mlp_data(500, 12)
    Pt = dev(P.astype(np.float32))
    m = torch.zeros(5313, device="cuda")
    v = torch.zeros(5313, device="cuda")
    P64 = P.astype(np.float32).astype(np.float64)
    m64, v64 = np.zeros(5313), np.zeros(5313)
    say("adam")
    for step in range(1, 4):
        A.mlp_train_step(Pt, m, v, dev(X), dev(y), step, 1e-3)
        _, g, _ = oracle.mlp_fwd_bwd(P64, X, y)
        oracle.adam_step(P64, g, m64, v64, step, lr=1e-3)
    torch.cuda.synchronize()
    # near-zero gradients are normalised by Adam: allow half a learning rate
    assert np.abs(Pt.cpu().numpy() - P64).max() <= 5e-4


def test_mlp_bf16_forward(A):
    # BF16 inference is one fixed FP32 computation: bit-identical to the oracle's
    P, X, _ = _mlp_data(700, 13)
    Pt = dev(P.astype(np.float32))
    say("mlp bf16")
    w = A.mlp_export_bf16(Pt)
    z = A.mlp_forward_bf16(w, dev(X))
    torch.cuda.synchronize()
    wb = w.cpu().numpy()
    assert (wb == oracle.bf16_encode(P.astype(np.float32))).all()
    rz = oracle.mlp_logits_bf16(wb, X)
    assert (z.cpu().numpy() == rz).all()


# ---------------------------------------------------------------- batch
def test_batch_matches_oracle_per_descriptor(A):
    x, adj = graph(1500, 32, 30, "int")
    nq = 400
    r = synth.rng(14)
    q = synth.small_int(15, nq, 32, hi=256)
    kind = (r.random(nq) < 0.5).astype(np.int32)
    kk = r.choice(np.array([1, 10, 100], np.int32), size=nq)
    ee = r.choice(np.array([0.0, 0.1, 0.2], np.float32), size=nq)
    vert = r.integers(0, 1500, size=nq).astype(np.int32)
    sv = np.where(kind == 1, vert, 0).astype(np.int32)
    rows = np.arange(nq, dtype=np.int64)
    descs, total, kmax = A.make_descs(kind, sv, rows, kk, ee)
    say("batch", nq, total, kmax)
    store = A.VectorStore(dev(x), "f32")
    g = A.DeviceGraph(dev(adj))
    ids, ds, st = A.search_batch(store, g, dev(q), descs, nq, total, kmax, queue_cap=BIG_L)
    torch.cuda.synchronize()
    ids, ds, st = ids.cpu().numpy(), ds.cpu().numpy(), st.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(kk)[:-1]])
    for i in range(nq):
        if kind[i] == 1:
            rid, rd, rst = oracle.range_search_indexed(x, adj, [vert[i]], int(kk[i]), float(ee[i]), cap_L=BIG_L)
        else:
            rid, rd, rst = oracle.range_search(x, adj, q[i:i + 1], [0], int(kk[i]), float(ee[i]), cap_L=BIG_L)
        sl = slice(off[i], off[i] + kk[i])
        assert ids[sl].tolist() == rid[0].tolist(), i
        assert (ds[sl] == rd[0]).all(), i
        assert st[i, 0] == rst[0, 0] and st[i, 1] == rst[0, 1], i


def test_batch_bad_descriptor_skipped(A):
    x, adj = graph(300, 16, 6, "int")
    kind = np.array([0, 0, 1, 0], np.int32)
    sv = np.array([0, 0, 5000, 0], np.int32)
    rows = np.array([0, 99, 0, 1], np.int64)   # row 99 is outside the 2 query rows
    kk = np.array([5, 5, 5, 5], np.int32)
    descs, total, kmax = A.make_descs(kind, sv, rows, kk, np.zeros(4, np.float32))
    say("batch bad")
    store = A.VectorStore(dev(x), "f32")
    g = A.DeviceGraph(dev(adj))
    ids, ds, st = A.search_batch(store, g, dev(synth.small_int(16, 2, 16, hi=256)), descs, 4, total, kmax)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert (st[[1, 2], 2] & A.FLAG_BAD_ID != 0).all()
    assert (st[[0, 3], 2] & A.FLAG_BAD_ID == 0).all()


# ---------------------------------------------------------------- trace and learned stop
def test_trace_rows_and_labels(A):
    x, adj = graph(1500, 32, 30, "int")
    q = synth.small_int(17, 200, 32, hi=256)
    rows, itv = 32, 2
    trace = torch.full((200 * rows * A.TRACE_W,), float("nan"), device="cuda")
    say("trace")
    store = A.VectorStore(dev(x), "f32")
    g = A.DeviceGraph(dev(adj))
    ids, ds, st = A.search(store, g, dev(q), dev(np.zeros((200, 1), np.int32)), 10, 0.1,
                           trace=trace, trace_rows=rows, trace_interval=itv)
    plain = A.search(store, g, dev(q), dev(np.zeros((200, 1), np.int32)), 10, 0.1)
    torch.cuda.synchronize()
    for u, v in zip((ids, ds, st), plain):
        assert (u.cpu().numpy() == v.cpu().numpy()).all()   # tracing does not change the search
    T = trace.cpu().numpy().reshape(200, rows, A.TRACE_W)
    hops = st.cpu().numpy()[:, 0]
    for i in range(200):
        n = min(rows, hops[i] // itv)
        lab = T[i, :, 16]
        assert (lab[n:] == -1).all() and np.isin(lab[:n], [0.0, 1.0]).all()
        assert (np.diff(lab[:n]) >= 0).all()             # once stable, stays stable
        assert np.isfinite(T[i, :n, :16]).all()
        assert (T[i, :n, 18] == itv * np.arange(1, n + 1)).all()


def test_learned_stop_extremes(A):
    x, adj = graph(1500, 32, 30, "int")
    q = synth.small_int(18, 100, 32, hi=256)
    store = A.VectorStore(dev(x), "f32")
    g = A.DeviceGraph(dev(adj))
    w = A.mlp_export_bf16(dev(np.zeros(5313, np.float32)))
    mean = torch.zeros(16, device="cuda")
    istd = torch.ones(16, device="cuda")
    seeds = dev(np.zeros((100, 1), np.int32))
    say("learned stop")
    plain = A.search(store, g, dev(q), seeds, 10, 0.1)
    never = A.search(store, g, dev(q), seeds, 10, 0.1, stop=A.StopModel(w, mean, istd, 1.0, 3))
    always = A.search(store, g, dev(q), seeds, 10, 0.1, stop=A.StopModel(w, mean, istd, 0.0, 3))
    torch.cuda.synchronize()
    for u, v in zip(plain, never):
        assert (u.cpu().numpy() == v.cpu().numpy()).all()
    sa = always[2].cpu().numpy()
    sp = plain[2].cpu().numpy()
    stopped = (sa[:, 2] & A.FLAG_LEARNED_STOP) != 0
    assert (sa[stopped, 0] == 3).all()
    assert (sa[~stopped, 0] == sp[~stopped, 0]).all() and (sp[~stopped, 0] < 3).all()
    # never before hop H, always from hop H on (H a checkpoint: a multiple of 3)
    H = 3 * int(np.median(sp[:, 0]) // 3)
    late = A.search(store, g, dev(q), seeds, 10, 0.1,
                    stop=A.StopModel(w, mean, istd, 1.0, 3, tau_long=0.0, long_hops=H))
    torch.cuda.synchronize()
    sl = late[2].cpu().numpy()
    long_q = sp[:, 0] >= H
    assert long_q.any() and (~long_q).any()
    assert (sl[long_q, 0] == H).all() and ((sl[long_q, 2] & A.FLAG_LEARNED_STOP) != 0).all()
    assert (sl[~long_q, 0] == sp[~long_q, 0]).all()
    assert (late[0].cpu().numpy()[~long_q] == plain[0].cpu().numpy()[~long_q]).all()


def test_hip_graph_capture_replays(A):
    """The persistent launch (counter reset kernel + search kernel, no memset) can be
    captured in a HIP graph; every replay, with eager work in between, matches eager."""
    x, adj = graph(1500, 32, 30, "int")
    q = synth.small_int(19, 300, 32, hi=256)
    store = A.VectorStore(dev(x), "bf16")
    g = A.DeviceGraph(dev(adj))
    Q = dev(q)
    seeds = dev(np.zeros((300, 1), np.int32))
    out = (torch.empty((300, 10), dtype=torch.int32, device="cuda"),
           torch.empty((300, 10), dtype=torch.float32, device="cuda"),
           torch.empty((300, 4), dtype=torch.int32, device="cuda"))
    say("graph capture")
    ref = [t.cpu().numpy() for t in A.search(store, g, Q, seeds, 10, 0.1)]
    A.search(store, g, Q, seeds, 10, 0.1, out=out)   # warm the workspace cache
    torch.cuda.synchronize()
    cg = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(cg, stream=s):
            A.search(store, g, Q, seeds, 10, 0.1, out=out)
    torch.cuda.synchronize()
    big = dev(synth.small_int(20, 4000, 32, hi=256))
    for rep in range(4):
        for t in out:
            t.fill_(-7)
        A.search(store, g, Q[:5], seeds[:5], 3, 0.0)       # unrelated eager work
        # eager work that needs a larger workspace than the captured one: the
        # captured buffer must stay allocated and untouched by it
        with torch.cuda.stream(s):
            A.search(store, g, big, dev(np.zeros((4000, 1), np.int32)), 100, 0.2, hash_slots=256)
        torch.cuda.synchronize()
        cg.replay()
        torch.cuda.synchronize()
        for u, v in zip(out, ref):
            assert (u.cpu().numpy() == v).all(), rep
