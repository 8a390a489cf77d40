"""CPU oracle for the DEG search path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, sequential C implementation (``deg_oracle.c``) of what the
paper's method computes, wrapped with ctypes. Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import this package; the HIP library
never does, and this package never imports the HIP library.

What it covers (each C function cites its passage):
  * distances: squared L2 and 1 - <x,q> in FP32 (fixed C32x4 order) and FP64
  * RangeSearch (Algorithm 1), plain and exploratory (query vertex excluded)
  * exact kNN in FP64 (Eq. knn), the ground truth for recall (Eq. recall@k)
  * incremental construction (Sec. 5.2, Algorithms 2-4) and continuous
    refinement (Algorithm 5); it builds every graph the GPU searches
  * the graph checker (Sec. 5.1: even-regular, undirected, loop-free,
    connected, bridgeless)
  * BF16 / FP8-e4m3 encoders and the FP64 MLP forward/backward
  * BF16 inference of the MLP: BF16 weights, the inputs of both hidden layers
    rounded to BF16 (nearest-even), wide accumulation
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "deg_oracle.c"
_LIB = _HERE / "liboracle.so"

L2, IP = 0, 1

# parameters of the incremental construction (Table "DEG parameters"):
# SIFT1M row (d=30, k_ext=60, eps_ext=0.2, k_opt=30, eps_opt=0.001, i_opt=5)
DEFAULT_BUILD = dict(k_ext=60, eps_ext=0.2, k_opt=30, eps_opt=0.001, i_opt=5)


def build(force: bool = True) -> Path:
    """Compile the oracle shared library with gcc (strict FP: no contraction)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        cmd = ["gcc", "-O3", "-mavx2", "-mfma", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-pthread", "-o", str(tmp), str(_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        _lib = C.CDLL(str(_LIB))
        _declare(_lib)
    return _lib


P = C.c_void_p
I32, I64, F32, U64, U8 = C.c_int32, C.c_int64, C.c_float, C.c_uint64, C.c_uint8


def _declare(L):
    L.or_dist32.restype = F32
    L.or_dist32.argtypes = [P, P, I64, I32]
    L.or_dist32_def.restype = F32
    L.or_dist32_def.argtypes = [P, P, I64, I32]
    L.or_dist64.restype = C.c_double
    L.or_dist64.argtypes = [P, P, I64, I32]
    L.or_range_search.restype = I32
    L.or_range_search.argtypes = [P, I64, I64, I64, I32, P, I32, I64, P, I64, I64, P, I32, P, P, P,
                                  P, P, I32, I32, F32, I64, I32, P, P, I64, I32, P, P, I64, P, I32]
    L.or_mlp_logit_bf16.restype = F32
    L.or_mlp_logit_bf16.argtypes = [P, P]
    L.or_mlp_logits_bf16_rows.argtypes = [P, P, I64, P]
    L.or_rerank.restype = I32
    L.or_rerank.argtypes = [P, I64, I64, I32, P, P, I32, I32, P, P]
    L.or_knn64.restype = I32
    L.or_knn64.argtypes = [P, I64, I64, I64, I32, P, I64, I64, I32, P, P, P, I32]
    L.or_graph_create.restype = P
    L.or_graph_create.argtypes = [P, I64, I64, I64, I32, I32]
    L.or_graph_free.argtypes = [P]
    L.or_graph_init.argtypes = [P]
    L.or_graph_extend.argtypes = [P, I64, I32, F32, I32, F32, I32, I32]
    L.or_graph_optimize_edge.argtypes = [P, I32, I32, I32, I32, F32]
    L.or_graph_refine.argtypes = [P, I64, U64, I32, I32, F32]
    L.or_graph_check_mrng.argtypes = [P, I32, I32]
    L.or_graph_nv.restype = I64
    L.or_graph_nv.argtypes = [P]
    L.or_graph_export.argtypes = [P, P, P, P]
    L.or_graph_import.argtypes = [P, P, P, P, I64]
    L.or_graph_counters.argtypes = [P, P]
    L.or_build.restype = I32
    L.or_build.argtypes = [P, I64, I64, I64, I32, I32, I32, F32, I32, F32, I32, I32, I64, U64, P, P,
                           P, I32]
    L.or_graph_extend_with.restype = I32
    L.or_graph_extend_with.argtypes = [P, I64, P, P, I64, I32, F32, I32, I32]
    L.or_build_batched.restype = I32
    L.or_build_batched.argtypes = [P, I64, I64, I64, I32, I32, I32, F32, I32, F32, I32, I32, I64,
                                   I32, P, P, P]
    L.or_build_block_size.restype = I64
    L.or_build_block_size.argtypes = [I64, I64, I64]
    L.or_check_graph.restype = I32
    L.or_check_graph.argtypes = [P, I64, I32, P, P, I64, I64, I32, P]
    L.or_bf16_encode.restype = C.c_uint16
    L.or_bf16_encode.argtypes = [F32]
    L.or_bf16_decode.restype = F32
    L.or_bf16_decode.argtypes = [C.c_uint16]
    L.or_e4m3_decode.restype = F32
    L.or_e4m3_decode.argtypes = [U8]
    L.or_e4m3_encode.restype = U8
    L.or_e4m3_encode.argtypes = [F32]
    L.or_fp8_encode_rows.argtypes = [P, I64, I64, I64, P, I64, P]
    L.or_fp8_decode_rows.argtypes = [P, I64, I64, I64, P, P, I64]
    L.or_bf16_encode_array.argtypes = [P, I64, P]
    L.or_mlp_nparams.restype = I32
    L.or_mlp_fwd_bwd.restype = I32
    L.or_mlp_fwd_bwd.argtypes = [P, P, P, I64, P, P, P]
    L.or_adam_step.argtypes = [P, P, P, P, I64, I64, C.c_double, C.c_double, C.c_double,
                               C.c_double]
    L.or_medoid.restype = I64
    L.or_medoid.argtypes = [P, I64, I64, I64, I32]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def nthreads_default():
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


# ---------------------------------------------------------------- distances
def dist32(x, q, metric=L2) -> float:
    x, q = _f32(x), _f32(q)
    return float(lib().or_dist32(_p(x), _p(q), x.shape[-1], metric))


def dist32_def(x, q, metric=L2) -> float:
    x, q = _f32(x), _f32(q)
    return float(lib().or_dist32_def(_p(x), _p(q), x.shape[-1], metric))


def dist64(x, q, metric=L2) -> float:
    x, q = _f32(x), _f32(q)
    return float(lib().or_dist64(_p(x), _p(q), x.shape[-1], metric))


# ---------------------------------------------------------------- search
class _OrStop(C.Structure):
    _fields_ = [("w", C.c_void_p), ("mean", C.c_void_p), ("istd", C.c_void_p),
                ("tau", C.c_float), ("tau_long", C.c_float), ("interval", C.c_int32),
                ("long_hops", C.c_int32)]


class StopModel:
    """Learned-stop parameters for the oracle's search: BF16 weights (5313 uint16
    bit patterns), the 16 feature means and inverse standard deviations, the
    probability threshold tau (tau_long from hop long_hops on) and the
    checkpoint interval."""

    def __init__(self, w_bf16, mean, inv_std, tau, interval, tau_long=None, long_hops=0):
        self.w = np.ascontiguousarray(w_bf16, np.uint16)
        self.mean = _f32(mean)
        self.istd = _f32(inv_std)
        assert self.w.shape == (5313,) and self.mean.shape == (16,) and self.istd.shape == (16,)
        self.tau, self.interval = float(tau), int(interval)
        self.tau_long = float(tau if tau_long is None else tau_long)
        self.long_hops = int(long_hops)

    def c(self):
        return _OrStop(self.w.ctypes.data, self.mean.ctypes.data, self.istd.ctypes.data,
                       self.tau, self.tau_long, self.interval, self.long_hops)


def _exclusion_csr(exclude, nq):
    """Per-query exclusion lists as CSR arrays: `exclude` is an (nq,) id array
    (one id per query, -1 = none) or a sequence of nq id lists."""
    if exclude is None:
        return None, None
    if isinstance(exclude, np.ndarray) and exclude.ndim == 1 and exclude.dtype != object:
        lists = [[int(v)] if v >= 0 else [] for v in exclude.tolist()]
    else:
        lists = [list(map(int, e)) for e in exclude]
    assert len(lists) == nq
    off = np.zeros(nq + 1, np.int64)
    off[1:] = np.cumsum([len(e) for e in lists])
    ids = np.array([v for e in lists for v in e] or [0], np.int32)
    return off, ids


def range_search(vec, adj, queries, seeds, k, eps, metric=L2, exclude=None, cap_L=0,
                 order_mode=0, k_arr=None, eps_arr=None, out_k=None, nthreads=None, k_pool=0,
                 kind=None, stop: StopModel | None = None, trace_rows=0, trace_interval=0):
    """RangeSearch (Algorithm 1) for every query row.

    seeds: (nq, ns) int32 or (ns,) shared by all queries.
    exclude: optional per-query ids kept out of the result, (nq,) or a list of lists
    (they still enter S and C).
    k_pool: R holds max(k, k_pool) entries; out_k of them are returned.
    kind: optional (nq,) 1 for exploratory queries (a stop feature).
    stop: optional learned stop; trace_rows > 0 also returns the trace rows
    (nq, trace_rows, 20).
    Returns ids (nq, out_k), dists (nq, out_k), stats (nq, 4) = hops, evals,
    max live |S|, flags (1 overflow, 16 learned stop) [, trace].
    """
    vec, queries, adj = _f32(vec), _f32(queries), _i32(adj)
    n, m = vec.shape
    nq = queries.shape[0]
    seeds = np.asarray(seeds, dtype=np.int32)
    if seeds.ndim == 1:
        seeds = np.broadcast_to(seeds, (nq, seeds.shape[0]))
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    ex_off, ex_ids = _exclusion_csr(exclude, nq)
    ka = None if k_arr is None else _i32(k_arr)
    ea = None if eps_arr is None else _f32(eps_arr)
    kd = None if kind is None else _i32(kind)
    ok = int(out_k or (int(ka.max()) if ka is not None else k))
    ids = np.empty((nq, ok), np.int32)
    ds = np.empty((nq, ok), np.float32)
    st = np.empty((nq, 4), np.int64)
    sc = None if stop is None else stop.c()
    tr = np.empty((nq, trace_rows, 20), np.float32) if trace_rows > 0 else None
    rc = lib().or_range_search(_p(vec), n, m, m, metric, _p(adj), adj.shape[1], adj.shape[1],
                               _p(queries), nq, m, _p(seeds), seeds.shape[1], _p(ex_off),
                               _p(ex_ids), _p(ka), _p(ea), _p(kd), int(k), int(k_pool),
                               float(eps), int(cap_L), int(order_mode),
                               None if sc is None else C.byref(sc), _p(tr), int(trace_rows),
                               int(trace_interval), _p(ids), _p(ds), ok, _p(st),
                               int(nthreads or nthreads_default()))
    if rc:
        raise ValueError("or_range_search: invalid arguments")
    return (ids, ds, st) if tr is None else (ids, ds, st, tr)


def range_search_indexed(vec, adj, qids, k, eps, metric=L2, query_vec=None, exclude=None, **kw):
    """Exploratory search: seed = the query's own vertex, which is kept out of R
    (with `exclude`, a list of lists, further ids are kept out too)."""
    qids = _i32(qids)
    qv = _f32(vec if query_vec is None else query_vec)[qids]
    ex = [[int(v)] for v in qids.tolist()] if exclude is None else \
        [[int(v)] + list(map(int, e)) for v, e in zip(qids.tolist(), exclude)]
    kw.setdefault("kind", np.ones(len(qids), np.int32))
    return range_search(vec, adj, qv, qids[:, None], k, eps, metric, exclude=ex, **kw)


def rerank(vec, q, pool, k, metric=L2):
    vec, q, pool = _f32(vec), _f32(q), _i32(pool)
    ids = np.empty(k, np.int32)
    ds = np.empty(k, np.float32)
    lib().or_rerank(_p(vec), vec.shape[1], vec.shape[1], metric, _p(q), _p(pool), pool.shape[0],
                    k, _p(ids), _p(ds))
    return ids, ds


def knn64(base, queries, k, metric=L2, exclude=None, nthreads=None):
    """Exact kNN by (FP64 distance, id). Returns ids (nq,k) int32, dists (nq,k) float64."""
    base, queries = _f32(base), _f32(queries)
    nq = queries.shape[0]
    ids = np.empty((nq, k), np.int32)
    ds = np.empty((nq, k), np.float64)
    ex = None if exclude is None else _i32(exclude)
    rc = lib().or_knn64(_p(base), base.shape[0], base.shape[1], base.shape[1], metric,
                        _p(queries), nq, queries.shape[1], k, _p(ex), _p(ids), _p(ds),
                        int(nthreads or nthreads_default()))
    if rc:
        raise ValueError("or_knn64: invalid arguments")
    return ids, ds


def medoid(vec, metric=L2) -> int:
    vec = _f32(vec)
    return int(lib().or_medoid(_p(vec), vec.shape[0], vec.shape[1], vec.shape[1], metric))


# ---------------------------------------------------------------- construction
class Graph:
    """Mutable DEG under construction (weights kept), for step-level tests."""

    def __init__(self, vec, d, metric=L2):
        self.vec = _f32(vec)
        self.n, self.m = self.vec.shape
        self.d = d
        self.h = lib().or_graph_create(_p(self.vec), self.n, self.m, self.m, metric, d)
        if not self.h:
            raise ValueError("invalid graph parameters (d even, >= 4, n >= d+1)")

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_graph_free(self.h)
            self.h = None

    def init(self):
        assert lib().or_graph_init(self.h) == 0

    def extend(self, v, k_ext=60, eps_ext=0.2, k_opt=30, eps_opt=0.001, i_opt=5, do_opt=True):
        return lib().or_graph_extend(self.h, v, k_ext, eps_ext, k_opt, eps_opt, i_opt,
                                     int(do_opt))

    def extend_with(self, v, ids, dists, k_opt=30, eps_opt=0.001, i_opt=5, do_opt=True):
        """The edits for vertex v given its search result (sorted ids and distances)."""
        ids, dists = _i32(ids), _f32(dists)
        return lib().or_graph_extend_with(self.h, v, _p(ids), _p(dists), len(ids), k_opt, eps_opt,
                                          i_opt, int(do_opt))

    def optimize_edge(self, v1, v2, i_opt=5, k_opt=30, eps_opt=0.001):
        return lib().or_graph_optimize_edge(self.h, v1, v2, i_opt, k_opt, eps_opt)

    def refine(self, rounds, seed=1, i_opt=5, k_opt=30, eps_opt=0.001):
        return lib().or_graph_refine(self.h, rounds, seed, i_opt, k_opt, eps_opt)

    def check_mrng(self, v1, v2):
        return bool(lib().or_graph_check_mrng(self.h, v1, v2))

    @property
    def nv(self):
        return int(lib().or_graph_nv(self.h))

    def export(self):
        adj = np.empty((self.n, self.d), np.int32)
        w = np.empty((self.n, self.d), np.float32)
        cnt = np.empty(self.n, np.int32)
        lib().or_graph_export(self.h, _p(adj), _p(w), _p(cnt))
        return adj, w, cnt

    def counters(self):
        c = np.zeros(8, np.int64)
        lib().or_graph_counters(self.h, _p(c))
        return dict(zip(["phase2", "opt_calls", "opt_commit", "opt_revert", "case_a", "case_b",
                         "searches", "err"], c.tolist()))


def build_graph(vec, d, metric=L2, k_ext=60, eps_ext=0.2, k_opt=30, eps_opt=0.001, i_opt=5,
                do_opt=True, refine_rounds=0, seed=1, verbose=0):
    """Incremental DEG construction of every vertex in id order (Sec. 5.2).

    Returns adjacency (n, d) int32, weights (n, d) float32 and build counters.
    """
    vec = _f32(vec)
    n, m = vec.shape
    adj = np.empty((n, d), np.int32)
    w = np.empty((n, d), np.float32)
    cnt = np.zeros(8, np.int64)
    rc = lib().or_build(_p(vec), n, m, m, metric, d, k_ext, eps_ext, k_opt, eps_opt, i_opt,
                        int(do_opt), refine_rounds, seed, _p(adj), _p(w), _p(cnt), verbose)
    if rc:
        raise RuntimeError("or_build failed (%d)" % rc)
    return adj, w, dict(zip(["phase2", "opt_calls", "opt_commit", "opt_revert", "case_a",
                             "case_b", "searches", "err"], cnt.tolist()))


def build_graph_batched(vec, d, batch, metric=L2, k_ext=60, eps_ext=0.2, k_opt=30, eps_opt=0.001,
                        i_opt=5, do_opt=True, lag=0):
    """Construction in blocks of at most `batch` vertices whose searches all run on
    the graph as it stands when the block starts; the edits then follow in id
    order (batch = 1 is the one-at-a-time build of Sec. 5.2). With lag = 1 the
    searches of a block run before the previous block's edits are applied.
    Returns adjacency, weights and counters like build_graph."""
    vec = _f32(vec)
    n, m = vec.shape
    adj = np.empty((n, d), np.int32)
    w = np.empty((n, d), np.float32)
    cnt = np.zeros(8, np.int64)
    rc = lib().or_build_batched(_p(vec), n, m, m, metric, d, k_ext, eps_ext, k_opt, eps_opt, i_opt,
                                int(do_opt), batch, int(lag), _p(adj), _p(w), _p(cnt))
    if rc:
        raise RuntimeError("or_build_batched failed (%d)" % rc)
    return adj, w, dict(zip(["phase2", "opt_calls", "opt_commit", "opt_revert", "case_a",
                             "case_b", "searches", "err"], cnt.tolist()))


def build_block_size(nv, batch, left) -> int:
    """Vertices in the next block of the batched build."""
    return int(lib().or_build_block_size(nv, batch, left))


def check_graph(adj, vec=None, w=None, metric=L2):
    """Graph invariants of Sec. 5.1. Returns a dict; 'flags' == 0 means all hold."""
    adj = _i32(adj)
    n, d = adj.shape
    out = np.zeros(6, np.int64)
    v = None if vec is None else _f32(vec)
    ww = None if w is None else _f32(w)
    lib().or_check_graph(_p(adj), n, d, _p(ww), _p(v), 0 if v is None else v.shape[1],
                         0 if v is None else v.shape[1], metric, _p(out))
    return dict(zip(["flags", "edges", "reached", "bridges", "indeg_min", "indeg_max"],
                    out.tolist()))


# ---------------------------------------------------------------- encodings
def bf16_encode(x):
    x = _f32(x)
    out = np.empty(x.shape, np.uint16)
    lib().or_bf16_encode_array(_p(x), x.size, _p(out))
    return out


def bf16_decode(h):
    return (np.asarray(h, np.uint16).astype(np.uint32) << 16).view(np.float32)


def e4m3_decode_table():
    return np.array([lib().or_e4m3_decode(c) for c in range(256)], np.float32)


def e4m3_encode(x):
    return np.array([lib().or_e4m3_encode(float(v)) for v in np.ravel(x)], np.uint8).reshape(
        np.shape(x))


def fp8_encode_rows(x, stride=None):
    x = _f32(x)
    n, m = x.shape
    cs = stride or m
    codes = np.empty((n, cs), np.uint8)
    scale = np.empty(n, np.float32)
    lib().or_fp8_encode_rows(_p(x), n, m, m, _p(codes), cs, _p(scale))
    return codes, scale


def fp8_decode_rows(codes, scale, m):
    codes = np.ascontiguousarray(codes, np.uint8)
    scale = _f32(scale)
    n, cs = codes.shape
    out = np.empty((n, m), np.float32)
    lib().or_fp8_decode_rows(_p(codes), n, m, cs, _p(scale), _p(out), m)
    return out


# ---------------------------------------------------------------- MLP
def mlp_nparams():
    return int(lib().or_mlp_nparams())


def mlp_fwd_bwd(params, X, y=None, want_grad=True):
    P64 = np.ascontiguousarray(params, np.float64)
    X = _f32(X)
    B = X.shape[0]
    yy = None if y is None else _f32(y)
    loss = np.zeros(1, np.float64)
    grad = np.zeros(P64.shape[0], np.float64) if (want_grad and y is not None) else None
    logits = np.empty(B, np.float64)
    lib().or_mlp_fwd_bwd(_p(P64), _p(X), _p(yy), B, _p(loss), _p(grad), _p(logits))
    return float(loss[0]), grad, logits


def adam_step(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(grad, np.float64)
    lib().or_adam_step(_p(params), _p(g), _p(m), _p(v), params.shape[0], t, lr, b1, b2, eps)


def mlp_logits_bf16(w_bf16, X):
    """Logits of the stop network with BF16 weights (5313 uint16 bit patterns)
    for rows of 16 standardised features: the FP32 definition of
    or_mlp_logit_bf16 (BF16 inputs and first hidden layer, fused multiply-adds
    in index order, a halving tree for the output layer)."""
    w = np.ascontiguousarray(w_bf16, np.uint16)
    assert w.shape == (5313,)
    X = _f32(X)
    out = np.empty(X.shape[0], np.float32)
    lib().or_mlp_logits_bf16_rows(_p(w), _p(X), X.shape[0], _p(out))
    return out
