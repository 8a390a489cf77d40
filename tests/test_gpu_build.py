"""GPU graph construction (Sec. 5.2, Algorithm 3 without optimizeEdge) with the
searches of each block batched on the device, against the oracle's batched
schedule: the same adjacency (row order included) and the same edge weights,
bit for bit, at the same block limit; batch = 1 against the oracle's
one-vertex-at-a-time build; and the graph invariants of Sec. 5.1."""
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


def gpu_build(A, x, d, k_ext, eps, batch, metric=oracle.L2, lag=0):
    store = A.VectorStore(torch.from_numpy(np.ascontiguousarray(x)).cuda(), "f32", metric)
    adj, w, cnt = A.build_graph(store, x, d, k_ext, eps, batch, lag=lag)
    torch.cuda.synchronize()
    return adj.cpu().numpy(), w, cnt


def check(adj, w, x, metric):
    chk = oracle.check_graph(adj, x, w, metric)
    n, d = adj.shape
    assert chk["flags"] == 0, chk
    assert chk["edges"] == n * d // 2 and chk["bridges"] == 0 and chk["reached"] == n


@pytest.mark.parametrize("n,m,d,batch,metric", [
    (600, 16, 10, 1, oracle.L2),      # the one-at-a-time schedule
    (1500, 24, 10, 16, oracle.L2),
    (1500, 24, 10, 4096, oracle.L2),  # blocks limited by nv / 8 only
    (1200, 20, 12, 64, oracle.IP),
    (2500, 33, 30, 256, oracle.L2),   # degree 30, ragged dimension
    (900, 16, 80, 64, oracle.L2),     # rows longer than a wave
])
def test_build_matches_oracle_schedule(A, n, m, d, batch, metric):
    x = synth.small_int(30 + d, n, m, hi=64) if metric == oracle.L2 else synth.small_unit(31, n, m)
    k_ext, eps = 2 * d, 0.2
    say("build", n, m, d, batch, metric)
    adj, w, cnt = gpu_build(A, x, d, k_ext, eps, batch, metric)
    assert cnt["lossy"] == 0 and cnt["searches"] == n - d - 1
    ra, rw, rc = oracle.build_graph_batched(x, d, batch, metric, k_ext=k_ext, eps_ext=eps,
                                            do_opt=False)
    assert (adj == ra).all(), "adjacency differs in %d rows" % int((adj != ra).any(1).sum())
    assert (w == rw).all()
    assert cnt["phase2"] == rc["phase2"]
    check(adj, w, x, metric)
    if batch == 1:
        sa, sw, _ = oracle.build_graph(x, d, metric, k_ext=k_ext, eps_ext=eps, do_opt=False)
        assert (adj == sa).all() and (w == sw).all()


@pytest.mark.parametrize("n,m,d,batch,metric", [
    (1500, 24, 10, 16, oracle.L2),
    (1200, 20, 12, 64, oracle.IP),
    (2500, 33, 30, 4096, oracle.L2),
])
def test_build_with_lag_matches_oracle_schedule(A, n, m, d, batch, metric):
    # a block searches before the previous block's edits (which the host applies
    # meanwhile): the oracle's lag-1 schedule, byte for byte
    x = synth.small_int(60 + d, n, m, hi=64) if metric == oracle.L2 else synth.small_unit(61, n, m)
    say("build lag 1", n, m, d, batch, metric)
    adj, w, cnt = gpu_build(A, x, d, 2 * d, 0.2, batch, metric, lag=1)
    assert cnt["lossy"] == 0 and cnt["searches"] == n - d - 1
    ra, rw, rc = oracle.build_graph_batched(x, d, batch, metric, k_ext=2 * d, eps_ext=0.2,
                                            do_opt=False, lag=1)
    assert (adj == ra).all(), "adjacency differs in %d rows" % int((adj != ra).any(1).sum())
    assert (w == rw).all()
    assert cnt["phase2"] == rc["phase2"]
    check(adj, w, x, metric)


def test_build_cfg2_subset(A):
    # 8,000 vectors of the 1M x 128 integer workload, degree 30, blocks of up to 1,000
    x = np.ascontiguousarray(synth.cfg2()[0][:8000])
    say("build cfg2 subset")
    adj, w, cnt = gpu_build(A, x, 30, 60, 0.2, 1000)
    assert cnt["lossy"] == 0
    ra, rw, _ = oracle.build_graph_batched(x, 30, 1000, oracle.L2, k_ext=60, eps_ext=0.2,
                                           do_opt=False)
    assert (adj == ra).all() and (w == rw).all()
    check(adj, w, x, oracle.L2)


def test_build_result_too_small_is_an_error(A):
    # k_ext = 2 cannot supply 10 neighbours: the call fails instead of building
    x = synth.small_int(40, 300, 8, hi=64)
    store = A.VectorStore(torch.from_numpy(x).cuda(), "f32", oracle.L2)
    with pytest.raises(A.DegError):
        A.build_graph(store, x, 10, 2, 0.0, 16)


def test_build_full_size_invariants(A):
    # all 1,000,000 x 128 vectors of the integer workload, degree 30, blocks of up to
    # 16,384: the graph of Sec. 5.1 (even-regular, undirected, no loops, connected, no
    # bridges) and every edge weight equal to the oracle's FP32 distance; no search
    # lost a candidate to the capacity of S
    x = np.ascontiguousarray(synth.cfg2()[0])
    say("build cfg2 full size")
    adj, w, cnt = gpu_build(A, x, 30, 60, 0.2, 16384)
    say("build cfg2 full size counters", cnt)
    assert cnt["lossy"] == 0 and cnt["searches"] == len(x) - 31
    check(adj, w, x, oracle.L2)
