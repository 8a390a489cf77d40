"""The C ABI library loads and exports every symbol include/deg.h declares,
and host-side argument checks reject bad calls without touching the GPU."""
import ctypes as C
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent


def _declared():
    hdr = (ROOT / "include" / "deg.h").read_text()
    return sorted(set(re.findall(r"\b(deg_[a-z0-9_]+)\s*\(", hdr)))


@pytest.fixture(scope="module")
def L():
    from paper_2307_10479_amd import api
    return api.load_library()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings(L):
    for code in range(5):
        assert L.deg_status_string(code)


def _vec_graph(api, n=100, dim=16, degree=6, dtype=0, metric=0, stride=None):
    v = api.DegVectors(0x100000, n, dim, stride or dim, dtype, metric, None, 0x200000, dim, 0)
    g = api.DegGraph(0x300000, n, degree, degree)
    return v, g


def test_argument_validation_rejects_before_any_gpu_call(L):
    from paper_2307_10479_amd import api
    P = C.c_void_p(0x400000)
    o = api.DegSearchOpts()

    def call(v, g, k=10, eps=0.1, ns=1, qs=16):
        return L.deg_search(C.byref(v), C.byref(g), P, 10, qs, P, ns, k, eps, C.byref(o), P, P,
                            None, P, 1 << 20, None)

    bad = []
    v, g = _vec_graph(api, degree=5)
    bad.append(call(v, g))                          # odd degree (Sec. 5.1)
    v, g = _vec_graph(api, degree=2)
    bad.append(call(v, g))                          # degree below 4
    v, g = _vec_graph(api, degree=130)
    bad.append(call(v, g))                          # degree above 128 (two parts of a wave)
    v, g = _vec_graph(api)
    bad.append(call(v, g, k=0))                     # k < 1
    bad.append(call(v, g, k=1025))                  # k above the supported maximum (1024)
    bad.append(call(v, g, eps=-0.5))                # negative range factor
    bad.append(call(v, g, eps=float("nan")))
    bad.append(call(v, g, ns=0))                    # no seed
    bad.append(call(v, g, qs=8))                    # query stride below dim
    v, g = _vec_graph(api, stride=18)
    bad.append(call(v, g))                          # row stride not a multiple of 4
    v, g = _vec_graph(api, dtype=2)
    bad.append(call(v, g))                          # FP8 without scales
    v, g = _vec_graph(api)
    g.n = 99
    bad.append(call(v, g))                          # vectors and graph disagree on N
    assert all(b == 1 for b in bad), bad
    v, g = _vec_graph(api, dim=2000, stride=2000)
    assert call(v, g) == 2                          # dimension beyond the kernels' range
    # rows longer than a wave: the plain search is accepted, trace rows (stop features)
    # are not
    o.trace = 0x400000
    o.trace_rows_per_query = 4
    o.trace_interval = 2
    v, g = _vec_graph(api, degree=80)
    assert call(v, g) == 2
    # the residency query answers 0 for arguments a search would reject
    v, g = _vec_graph(api, degree=5)
    assert L.deg_search_resident_waves(C.byref(v), C.byref(g), 10, C.byref(o)) == 0
    v, g = _vec_graph(api)
    assert L.deg_search_resident_waves(C.byref(v), C.byref(g), 0, C.byref(o)) == 0


def test_build_argument_validation(L):
    from paper_2307_10479_amd import api
    P = C.c_void_p(0x400000)

    def call(degree=10, k_ext=20, eps=0.2, batch=64, dtype=0, n=100, dim=16, stride=16, hstride=16,
             lag=0):
        v = api.DegVectors()
        v.data, v.n, v.dim, v.row_stride, v.dtype, v.metric = P, n, dim, stride, dtype, 0
        p = api.DegBuildParams(degree=degree, k_ext=k_ext, eps_ext=eps, lag=lag, batch=batch)
        return L.deg_build_graph(C.byref(v), P, hstride, C.byref(p), P, None, None, None)

    bad = [call(degree=5), call(degree=2), call(degree=130), call(k_ext=0), call(k_ext=2000),
           call(eps=-1.0), call(eps=float("nan")), call(batch=0), call(dtype=1), call(n=10),
           call(hstride=8), call(lag=2), call(lag=-1)]
    assert all(b == 1 for b in bad), bad


def test_mrng_check_argument_validation(L):
    from paper_2307_10479_amd import api
    P = C.c_void_p(0x400000)
    g = api.DegGraph(0x400000, 100, 10, 10)
    assert L.deg_graph_check_mrng(None, P, 10, P, None, None, None) == 1
    assert L.deg_graph_check_mrng(C.byref(g), None, 10, P, None, None, None) == 1
    assert L.deg_graph_check_mrng(C.byref(g), P, 8, P, None, None, None) == 1  # rows too short
    g = api.DegGraph(0x400000, 100, 130, 130)
    assert L.deg_graph_check_mrng(C.byref(g), P, 130, P, None, None, None) == 1  # degree > 128


def test_knn_and_mlp_argument_validation(L):
    P = C.c_void_p(0x400000)
    assert L.deg_knn_bruteforce(P, 100, 16, 15, P, 10, 16, 10, 0, None, P, P, P, 1 << 20, None) == 1
    assert L.deg_knn_bruteforce(P, 100, 16, 16, P, 10, 16, 0, 0, None, P, P, P, 1 << 20, None) == 1
    assert L.deg_knn_bruteforce(P, 100, 16, 16, P, 10, 16, 10, 7, None, P, P, P, 1 << 20, None) == 1
    assert L.deg_mlp_train_step(P, P, P, P, P, 0, 1, 0.1, None, None, P, 1 << 20, None) == 1
    assert L.deg_mlp_train_step(P, P, P, P, P, 64, 0, 0.1, None, None, P, 1 << 20, None) == 1
    assert L.deg_medoid(P, 0, 16, 16, 0, P, P, 1 << 20, None) == 1
