"""GPU MRNG conformity of every edge (Algorithm 2, the selection step of
Algorithm 5) against the oracle's checkMRNG, edge by edge: on small graphs
built by the oracle (with and without optimizeEdge, L2 and IP, degree up to 80)
and on sampled vertices of the 1M x 128 graph of the batched GPU construction."""
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


def oracle_flags(x, adj, w, metric, vertices):
    n, d = adj.shape
    g = oracle.Graph(x, d, metric)
    cnt = (adj >= 0).sum(1).astype(np.int32)
    oracle.lib().or_graph_import(g.h, oracle._p(np.ascontiguousarray(adj, np.int32)),
                                 oracle._p(np.ascontiguousarray(w, np.float32)), oracle._p(cnt), n)
    out = np.full((len(vertices), d), 255, np.uint8)
    for i, v in enumerate(vertices):
        for j in range(d):
            if adj[v, j] >= 0:
                out[i, j] = 1 if g.check_mrng(int(v), int(adj[v, j])) else 0
    return out


def gpu_flags(A, adj, w, with_longest=False):
    G = A.DeviceGraph(torch.from_numpy(np.ascontiguousarray(adj)).cuda())
    ok, cnt, longest = A.check_mrng(G, torch.from_numpy(np.ascontiguousarray(w)).cuda())
    torch.cuda.synchronize()
    if with_longest:
        return ok.cpu().numpy(), int(cnt.item()), longest.cpu().numpy()
    return ok.cpu().numpy(), int(cnt.item())


def longest_by_definition(adj, w):
    # the largest weight of the row; equal weights: the smaller neighbour id
    out = np.full(len(adj), -1, np.int32)
    for v in range(len(adj)):
        live = [j for j in range(adj.shape[1]) if adj[v, j] >= 0]
        if live:
            out[v] = max(live, key=lambda j: (float(w[v, j]), -int(adj[v, j])))
    return out


@pytest.mark.parametrize("n,m,d,metric,do_opt", [
    (1500, 24, 10, oracle.L2, True),
    (1500, 24, 10, oracle.L2, False),
    (1200, 20, 12, oracle.IP, True),
    (900, 16, 80, oracle.L2, False),  # rows longer than a wave
])
def test_mrng_flags_match_oracle(A, n, m, d, metric, do_opt):
    x = synth.small_int(50 + d, n, m, hi=64) if metric == oracle.L2 else synth.small_unit(51, n, m)
    adj, w, _ = oracle.build_graph(x, d, metric, k_ext=2 * d, eps_ext=0.2, k_opt=d, do_opt=do_opt)
    say("mrng", n, m, d, metric, do_opt)
    ok, nfail, longest = gpu_flags(A, adj, w, with_longest=True)
    ref = oracle_flags(x, adj, w, metric, np.arange(n))
    assert (ok == ref).all(), "%d entries differ" % int((ok != ref).sum())
    assert (longest == longest_by_definition(adj, w)).all()
    assert nfail == int((ref == 0).sum())
    assert 0 < nfail < n * d  # both outcomes occur


def test_mrng_empty_slots_and_planted_failure(A):
    # a triangle (0, 1, 2) whose edge (0, 1) is longer than both other sides fails;
    # empty slots report 255
    adj = np.array([[1, 2, -1, -1], [0, 2, -1, -1], [0, 1, -1, -1]], np.int32)
    w = np.array([[5, 1, 0, 0], [5, 2, 0, 0], [1, 2, 0, 0]], np.float32)
    ok, nfail, longest = gpu_flags(A, adj, w, with_longest=True)
    assert longest.tolist() == [0, 0, 1]
    assert ok[:, 2:].tolist() == [[255, 255]] * 3
    assert ok[0, 0] == 0 and ok[1, 0] == 0  # (0, 1) from both ends
    assert ok[0, 1] == 1 and ok[2, 0] == 1 and ok[1, 1] == 1 and ok[2, 1] == 1
    assert nfail == 2


def test_mrng_full_size_sampled(A):
    x = np.ascontiguousarray(synth.cfg2()[0])
    store = A.VectorStore(torch.from_numpy(x).cuda(), "f32", oracle.L2)
    adj_t, w, _ = A.build_graph(store, x, 30, 60, 0.2, 16384)
    torch.cuda.synchronize()
    adj = adj_t.cpu().numpy()
    say("mrng full size")
    ok, nfail = gpu_flags(A, adj, w)
    sample = synth.rng(83).choice(len(x), size=2000, replace=False)
    ref = oracle_flags(x, adj, w, oracle.L2, sample)
    assert (ok[sample] == ref).all()
    assert nfail == int((ok == 0).sum())
    say("mrng full size: %.4f of the edge entries fail" % (nfail / ok.size))
