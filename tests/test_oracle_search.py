"""Pins of the oracle's distances and RangeSearch (Algorithm 1) against facts
the paper and the mathematics fix: a hand-traced example, exhaustive search
equals the exact kNN, the complete graph K_{d+1}, order independence, the
capacity bound, exploratory exclusion and recall."""
import json
from pathlib import Path

import numpy as np
import pytest

import oracle
import synth

GOLD = Path(__file__).resolve().parent / "golden"


# ---------------------------------------------------------------- distances
def test_dist32_integer_exact_vs_fp64():
    # integer values below 256 in 128 dims: every partial sum is an integer < 2^24
    x = synth.small_int(1, 200, 128, hi=256)
    q = synth.small_int(2, 1, 128, hi=256)[0]
    for i in range(200):
        d32 = oracle.dist32(x[i], q, oracle.L2)
        d64 = oracle.dist64(x[i], q, oracle.L2)
        assert d32 == d64 == float(((x[i].astype(np.int64) - q.astype(np.int64)) ** 2).sum())
        ip32 = oracle.dist32(x[i], q, oracle.IP)
        assert ip32 == np.float32(1.0 - float((x[i].astype(np.int64) * q.astype(np.int64)).sum()))


@pytest.mark.parametrize("m", [1, 3, 4, 5, 31, 100, 127, 128, 129, 300, 1369])
def test_dist32_vectorised_equals_definition(m):
    x = synth.small_float(m, 40, m)
    q = synth.small_float(m + 7, 1, m)[0]
    for metric in (oracle.L2, oracle.IP):
        for i in range(40):
            assert oracle.dist32(x[i], q, metric) == oracle.dist32_def(x[i], q, metric)


@pytest.mark.parametrize("m", [100, 128, 300, 1369])
def test_dist32_error_bound(m):
    # |fl32 - exact| <= gamma * sum |terms| with a fixed tree of depth <= m/128*4 + 5
    x = synth.small_float(10 + m, 50, m)
    q = synth.small_float(11 + m, 1, m)[0]
    depth = 4 * ((m + 127) // 128) + 5
    u = 2.0 ** -24
    for i in range(50):
        d64 = oracle.dist64(x[i], q, oracle.L2)
        d32 = oracle.dist32(x[i], q, oracle.L2)
        # the FP32 differences x-q are rounded once more: relative 2u per term
        assert abs(d32 - d64) <= (depth + 3) * u * d64 * 1.01
        s = float(np.dot(x[i].astype(np.float64), q.astype(np.float64)))
        a = float(np.dot(np.abs(x[i]).astype(np.float64), np.abs(q).astype(np.float64)))
        ip = oracle.dist32(x[i], q, oracle.IP)
        assert abs(ip - (1.0 - s)) <= (depth + 2) * u * (a + 1.0)


def test_dist_ip_is_one_minus_dot():
    x = np.array([[0.6, 0.8, 0.0, 0.0]], np.float32)
    q = np.array([0.8, 0.6, 0.0, 0.0], np.float32)
    assert abs(oracle.dist64(x[0], q, oracle.IP) - (1.0 - 0.96)) < 1e-7
    assert oracle.dist64(x[0], x[0], oracle.IP) == pytest.approx(0.0, abs=1e-7)


# ---------------------------------------------------------------- hand trace
def _toy():
    g = json.loads((GOLD / "alg1_toy.json").read_text())
    return np.array(g["adj"], np.int32), g["cases"]


def test_golden_hand_trace():
    adj, cases = _toy()
    for c in cases:
        pts = np.array(c["points"], np.float32).reshape(-1, 1)
        if "query_vertex" in c:
            ids, ds, st = oracle.range_search_indexed(pts, adj, [c["query_vertex"]], c["k"], c["eps"])
        else:
            q = np.array([[c["query"]]], np.float32)
            ids, ds, st = oracle.range_search(pts, adj, q, np.array([c["seeds"]]), c["k"], c["eps"])
        assert ids[0].tolist() == c["ids"], c["trace"]
        assert ds[0].tolist() == [float(v) for v in c["dists"]]
        assert st[0, 0] == c["hops"] and st[0, 1] == c["evals"], c["trace"]


def test_hand_trace_row_orders():
    adj, cases = _toy()
    for c in cases:
        if "query_vertex" in c:
            continue
        pts = np.array(c["points"], np.float32).reshape(-1, 1)
        q = np.array([[c["query"]]], np.float32)
        for mode in (1, 2):
            ids, ds, st = oracle.range_search(pts, adj, q, np.array([c["seeds"]]), c["k"], c["eps"],
                                              order_mode=mode)
            assert ids[0].tolist() == c["ids"] and st[0, 0] == c["hops"] and st[0, 1] == c["evals"]


# ---------------------------------------------------------------- graphs for the tests
_GRAPHS = {}


def built(n, m, d, kind="int", metric=oracle.L2, seed=0):
    key = (n, m, d, kind, metric, seed)
    if key not in _GRAPHS:
        if kind == "int":
            x = synth.small_int(seed, n, m, hi=64)
        elif kind == "unit":
            x = synth.small_unit(seed, n, m)
        else:
            x = synth.small_float(seed, n, m)
        adj, w, _ = oracle.build_graph(x, d, metric, k_ext=2 * d, eps_ext=0.2, k_opt=d,
                                       eps_opt=0.001, i_opt=5)
        _GRAPHS[key] = (x, adj, w)
    return _GRAPHS[key]


def brute_c32(x, q, k, metric, exclude=None):
    """(distance, id) top-k with the oracle's FP32 distance, by a full sort."""
    out = []
    for qi in range(q.shape[0]):
        d = [(oracle.dist32(x[i], q[qi], metric), i) for i in range(x.shape[0])
             if exclude is None or i != exclude[qi]]
        d.sort()
        out.append([i for _, i in d[:k]])
    return np.array(out)


@pytest.mark.parametrize("metric,kind", [(oracle.L2, "int"), (oracle.L2, "float"), (oracle.IP, "unit")])
def test_exhaustive_search_is_exact_knn(metric, kind):
    x, adj, _ = built(300, 16, 6, kind, metric)
    q = (synth.small_int(77, 20, 16, hi=64) if kind == "int" else
         synth.small_unit(77, 20, 16) if kind == "unit" else synth.small_float(77, 20, 16))
    for k in (1, 10, 40):
        ids, ds, st = oracle.range_search(x, adj, q, [0], k, float("inf"), metric)
        assert (st[:, 1] == x.shape[0]).all()  # every vertex evaluated exactly once
        assert (ids == brute_c32(x, q, k, metric)).all()


def test_complete_graph_exact_for_any_eps():
    d = 8
    x = synth.small_int(5, d + 1, 12, hi=8)  # many exact ties
    adj, w, _ = oracle.build_graph(x, d)
    assert oracle.check_graph(adj, x, w)["flags"] == 0
    q = synth.small_int(6, 30, 12, hi=8)
    for eps in (0.0, 0.1, 1.0):
        for seed in range(d + 1):
            ids, _, st = oracle.range_search(x, adj, q, [seed], 4, eps)
            assert (ids == brute_c32(x, q, 4, oracle.L2)).all()
            assert (st[:, 1] == d + 1).all()


@pytest.mark.parametrize("eps", [0.0, 0.1, 0.3])
def test_order_independence(eps):
    x, adj, _ = built(2000, 24, 30)
    q = synth.small_int(99, 100, 24, hi=64)
    base = oracle.range_search(x, adj, q, [0], 10, eps)
    for mode in (1, 2):
        ids, ds, st = oracle.range_search(x, adj, q, [0], 10, eps, order_mode=mode)
        assert (ids == base[0]).all() and (ds == base[1]).all()
        assert (st[:, :2] == base[2][:, :2]).all()


def test_capacity_hand_trace():
    # alg1_toy case 1 with L = 1: after hop 1 S keeps only 3 (1); pushing 4 (9)
    # into the full S evicts it, and 4 is within the end-of-hop range 9 -> overflow.
    # Hop 2 expands 3 (1 checked, out of range); S is empty: 2 hops, not 3.
    adj, cases = _toy()
    c = cases[0]
    pts = np.array(c["points"], np.float32).reshape(-1, 1)
    ids, ds, st = oracle.range_search(pts, adj, np.array([[7.0]], np.float32), [0], 2, 0.0, cap_L=1)
    assert ids[0].tolist() == [3, 4] and ds[0].tolist() == [1.0, 9.0]
    assert st[0, 0] == 2 and st[0, 1] == 6 and st[0, 3] & 1


def greedy_walk(x, adj, q, seed, k, eps):
    """Algorithm 1 with room for one candidate, stated as a walk: from the current
    vertex, check its unchecked neighbours, keep the k best vertices seen, and
    move to the closest new neighbour if it lies within the range r(1+eps)
    measured after the row; otherwise stop. r is the k-th best distance once
    more than k vertices were accepted, else infinite."""
    d = lambda i: np.float32(oracle.dist32(x[i], q))
    onep = np.float32(1.0) + np.float32(eps)
    R, full = [(d(seed), seed)], False

    def thr():
        return np.float32(R[k - 1][0]) * onep if full else np.float32(np.inf)

    checked = {seed}
    cur, hops = R[0], 0
    while True:
        hops += 1
        new = [n for n in adj[cur[1]].tolist() if n not in checked]
        checked.update(new)
        cand = [(d(n), n) for n in new]
        for e in cand:
            if not full or e[0] <= R[k - 1][0]:
                R = sorted(R + [e])
                if len(R) > k:
                    R, full = R[:k], True
        live = [e for e in cand if e[0] <= thr()]
        if not live:
            break
        cur = min(live)
    return [i for _, i in R], hops


def test_capacity_one_is_a_greedy_walk():
    x, adj, _ = built(2000, 24, 30)
    q = synth.small_int(91, 60, 24, hi=64)
    for k, eps in ((1, 0.0), (5, 0.1), (10, 0.3)):
        ids, ds, st = oracle.range_search(x, adj, q, [0], k, eps, cap_L=1)
        for i in range(q.shape[0]):
            gi, gh = greedy_walk(x, adj, q[i], 0, k, eps)
            assert ids[i].tolist() == gi + [-1] * (k - len(gi)), (k, eps, i)
            assert st[i, 0] == gh, (k, eps, i)


@pytest.mark.parametrize("L", [2, 8, 24])
def test_binding_capacity_is_order_independent(L):
    # per-push eviction of the largest keeps the L smallest of each row's
    # survivors whatever the order of the row: ids, counters and flags agree
    x, adj, _ = built(2000, 24, 30)
    q = synth.small_int(92, 100, 24, hi=64)
    base = oracle.range_search(x, adj, q, [0], 10, 0.2, cap_L=L)
    assert (base[2][:, 3] & 1).any()
    for mode in (1, 2):
        ids, ds, st = oracle.range_search(x, adj, q, [0], 10, 0.2, cap_L=L, order_mode=mode)
        assert (ids == base[0]).all() and (ds == base[1]).all()
        assert (st[:, :2] == base[2][:, :2]).all() and (st[:, 3] == base[2][:, 3]).all()


def test_unflagged_queries_equal_the_unbounded_search():
    # no live candidate lost <=> the bounded search is Algorithm 1 exactly
    x, adj, _ = built(2000, 24, 30)
    q = synth.small_int(93, 200, 24, hi=64)
    ref = oracle.range_search(x, adj, q, [0], 20, 0.2)
    mixed = 0
    for L in (40, 56, 64, 72, 128):
        ids, ds, st = oracle.range_search(x, adj, q, [0], 20, 0.2, cap_L=L)
        ok = (st[:, 3] & 1) == 0
        mixed += ok.any() and (~ok).any()
        assert (ids[ok] == ref[0][ok]).all() and (st[ok, :2] == ref[2][ok, :2]).all()
        # at a tight capacity the lost live entries change the work of most queries
        if L == 40:
            diff = (ids[~ok] != ref[0][~ok]).any(1) | (st[~ok, :2] != ref[2][~ok, :2]).any(1)
            assert diff.mean() > 0.5
    assert mixed >= 2


def test_capacity_bound_equals_unbounded():
    x, adj, _ = built(2000, 24, 30)
    q = synth.small_int(98, 100, 24, hi=64)
    ids0, ds0, st0 = oracle.range_search(x, adj, q, [0], 20, 0.2)
    L = int(st0[:, 2].max())
    ids1, ds1, st1 = oracle.range_search(x, adj, q, [0], 20, 0.2, cap_L=L)
    assert (ids0 == ids1).all() and (st0[:, :2] == st1[:, :2]).all() and (st1[:, 3] == 0).all()
    # a too-small capacity drops live candidates and is reported
    _, _, st2 = oracle.range_search(x, adj, q, [0], 20, 0.2, cap_L=8)
    assert (st2[:, 3] & 1).any()


# ---------------------------------------------------------------- FP32 rerank
def test_rerank_of_every_vertex_is_the_exact_knn():
    # integer data: FP32 distances are exact integers, so the rerank of a pool
    # holding all N vertices is the exact (distance, id) top-k
    x = synth.small_int(40, 700, 32, hi=256)
    q = synth.small_int(41, 12, 32, hi=256)
    pool = np.arange(700, dtype=np.int32)
    for i in range(12):
        d = ((x.astype(np.int64) - q[i].astype(np.int64)) ** 2).sum(1)
        order = np.lexsort((np.arange(700), d))[:15]
        ids, ds = oracle.rerank(x, q[i], pool[::-1].copy(), 15)
        assert ids.tolist() == order.tolist()
        assert ds.tolist() == d[order].astype(np.float64).tolist()
    # fewer candidates than k: padded; negative ids are not candidates
    ids, ds = oracle.rerank(x, q[0], np.array([5, -1, 3], np.int32), 4)
    assert ids[2:].tolist() == [-1, -1] and np.isinf(ds[2:]).all()
    assert sorted(ids[:2].tolist()) == [3, 5]


def test_rerank_ip_orders_by_one_minus_dot():
    u = synth.small_unit(42, 300, 16)
    q = synth.small_unit(43, 1, 16)[0]
    ids, ds = oracle.rerank(u, q, np.arange(300, dtype=np.int32), 5, oracle.IP)
    dots = u.astype(np.float64) @ q.astype(np.float64)
    assert ids[0] == int(np.argmax(dots))
    assert np.allclose(ds, 1.0 - dots[ids], atol=1e-6)


# ---------------------------------------------------------------- exclusion lists
def test_exclusion_lists_exhaustive_equal_brute_force_over_the_rest():
    # excluded ids enter S and C but never R: with eps = inf every vertex is
    # checked, so R is the exact top-k of the vertices not excluded
    x, adj, _ = built(300, 16, 6)
    q = synth.small_int(44, 10, 16, hi=64)
    r = synth.rng(45)
    ex = [r.choice(300, size=r.integers(0, 40), replace=False).tolist() for _ in range(10)]
    ids, ds, st = oracle.range_search(x, adj, q, [0], 12, float("inf"), exclude=ex)
    for i in range(10):
        keep = [j for j in range(300) if j not in set(ex[i])]
        d = [(oracle.dist32(x[j], q[i]), j) for j in keep]
        d.sort()
        assert ids[i].tolist() == [j for _, j in d[:12]]
        assert st[i, 1] == 300


def test_multi_seed_and_dedup():
    x, adj, _ = built(2000, 24, 30)
    q = synth.small_int(97, 30, 24, hi=64)
    seeds = np.tile(np.array([0, 17, 512], np.int32), (30, 1))
    ids, ds, st = oracle.range_search(x, adj, q, seeds, 10, 0.1)
    assert (st[:, 1] >= 3).all()
    for r in range(30):
        assert len(set(ids[r].tolist())) == 10


def test_indexed_excludes_query_vertex_and_is_exact_when_exhaustive():
    x, adj, _ = built(300, 16, 6)
    qids = np.arange(0, 300, 7, dtype=np.int32)
    ids, ds, st = oracle.range_search_indexed(x, adj, qids, 10, float("inf"))
    assert not (ids == qids[:, None]).any()
    assert (ids == brute_c32(x, x[qids], 10, oracle.L2, exclude=qids)).all()
    # duplicates of the query vector at distance 0 are allowed in the answer
    xd = x.copy()
    xd[5] = xd[3]
    ids, ds, _ = oracle.range_search_indexed(xd, adj, [3], 5, float("inf"))
    assert 5 in ids[0].tolist() and 3 not in ids[0].tolist() and ds[0, 0] == 0.0


def test_fewer_than_k_pads():
    d = 4
    x = synth.small_int(8, d + 1, 4, hi=10)
    adj, _, _ = oracle.build_graph(x, d)
    ids, ds, _ = oracle.range_search(x, adj, x[:1], [0], 8, 0.0)
    assert (ids[0, 5:] == -1).all() and np.isinf(ds[0, 5:]).all()
    ids, ds, _ = oracle.range_search_indexed(x, adj, [2], 8, 0.0)
    assert (ids[0, 4:] == -1).all() and 2 not in ids[0].tolist()


def test_knn64_brute_force():
    x = synth.small_float(3, 500, 10)
    q = synth.small_float(4, 20, 10)
    ids, ds = oracle.knn64(x, q, 7)
    for i in range(20):
        d = ((x.astype(np.float64) - q[i].astype(np.float64)) ** 2).sum(1)
        order = np.lexsort((np.arange(500), d))[:7]
        assert ids[i].tolist() == order.tolist()
        assert np.allclose(ds[i], d[order], rtol=0, atol=1e-12)
    ex = ids[:, 0].copy()
    ids2, _ = oracle.knn64(x, q, 7, exclude=ex)
    assert (ids2[:, :6] == ids[:, 1:]).all()


def test_medoid():
    x = np.array([[0, 0], [10, 0], [0, 10], [4, 5], [5, 4]], np.float32)
    # mean (3.8, 3.8): (4,5) and (5,4) are at the same distance; the smaller id wins
    assert oracle.medoid(x) == 3
    u = synth.small_unit(3, 200, 8)
    mean = u.astype(np.float64).mean(0)
    assert oracle.medoid(u, oracle.IP) == int(np.argmax(u.astype(np.float64) @ mean))
