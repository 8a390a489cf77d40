"""deg_search_noalloc (no workspace; the library's per-GPU scratch array)
against deg_search: the same ids, distances and counters, on two calls in a
row, the second with a smaller input, and on a search whose visited sets need
the shared tables (more queries than shared tables)."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def A():
    from paper_2307_10479_amd import api
    api.lib()
    return api


def _same(a, b, what):
    for u, v in zip(a, b):
        assert (u.cpu().numpy() == v.cpu().numpy()).all(), what


def test_noalloc_equals_search_on_two_calls(A):
    x = synth.small_int(50, 2000, 32, hi=64)
    adj, _, _ = oracle.build_graph(x, 16, k_ext=32, eps_ext=0.2, k_opt=16)
    store = A.VectorStore(dev(x), "f32")
    g = A.DeviceGraph(dev(adj))
    for nq, k, eps in ((700, 20, 0.2), (90, 5, 0.05)):
        q = dev(synth.small_int(51 + nq, nq, 32, hi=64))
        seeds = dev(np.zeros((nq, 1), np.int32))
        say("noalloc", nq, k, eps)
        ref = A.search(store, g, q, seeds, k, eps, queue_cap=512, hash_slots=256)
        got = A.search_noalloc(store, g, q, seeds, k, eps, queue_cap=512, hash_slots=256)
        torch.cuda.synchronize()
        _same(got, ref, "noalloc nq=%d" % nq)


def test_noalloc_with_shared_visited_tables(A):
    # eps = inf on a connected 60,000-vertex circulant graph: every query checks
    # all vertices, beyond the one table per wave, so all 16 queries need one
    # of the (at most 4) shared tables
    n = 60_000
    x = synth.small_float(52, n, 4)
    off = [1, -1, 2, -2, 3, -3, 4, -4]
    adj = ((np.arange(n)[:, None] + np.array(off)[None, :]) % n).astype(np.int32)
    store = A.VectorStore(dev(x), "f32")
    g = A.DeviceGraph(dev(adj))
    for nq in (16, 5):
        q = dev(synth.small_float(53 + nq, nq, 4))
        seeds = dev(np.zeros((nq, 1), np.int32))
        say("noalloc shared tables", nq)
        ref = A.search(store, g, q, seeds, 10, float("inf"), queue_cap=256, hash_slots=256)
        got = A.search_noalloc(store, g, q, seeds, 10, float("inf"), queue_cap=256,
                               hash_slots=256)
        torch.cuda.synchronize()
        _same(got, ref, "noalloc shared nq=%d" % nq)
        assert (got[2].cpu().numpy()[:, 1] == n).all()
