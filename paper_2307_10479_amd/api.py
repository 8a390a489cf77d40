"""Python binding of libdeg.so (ctypes): argument marshalling only.

Every step of the search runs in the library's HIP kernels; this module only
turns torch tensors (device memory, streams) into the C ABI's pointers and
sizes. It fails loudly when the library is not built or no GPU is present.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import torch

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libdeg.so"

L2, IP = 0, 1
F32, BF16, FP8 = 0, 1, 2
DTYPES = {"f32": F32, "bf16": BF16, "fp8": FP8}

FLAG_QUEUE_OVERFLOW = 1
FLAG_HASH_SPILL = 2
FLAG_HASH_FULL = 4
FLAG_BAD_ID = 8
FLAG_LEARNED_STOP = 16

MLP_NPARAMS = 5313
NFEAT = 16
TRACE_W = 20

STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported configuration",
          3: "workspace missing or too small", 4: "HIP runtime error"}


class DegError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__("%s failed: %s (%d)" % (fn, STATUS.get(code, "?"), code))
        self.code = code


class DegVectors(C.Structure):
    _fields_ = [("data", C.c_void_p), ("n", C.c_int64), ("dim", C.c_int32),
                ("row_stride", C.c_int32), ("dtype", C.c_int32), ("metric", C.c_int32),
                ("scale", C.c_void_p), ("f32_data", C.c_void_p), ("f32_stride", C.c_int32),
                ("reserved", C.c_int32)]


class DegGraph(C.Structure):
    _fields_ = [("adj", C.c_void_p), ("n", C.c_int64), ("degree", C.c_int32),
                ("row_stride", C.c_int32)]


class DegStopModel(C.Structure):
    _fields_ = [("weights_bf16", C.c_void_p), ("feat_mean", C.c_void_p),
                ("feat_inv_std", C.c_void_p), ("tau", C.c_float), ("interval", C.c_int32),
                ("tau_long", C.c_float), ("long_hops", C.c_int32)]


class DegSearchOpts(C.Structure):
    _fields_ = [("queue_cap", C.c_int32), ("hash_slots", C.c_int32), ("k_pool", C.c_int32),
                ("rerank", C.c_int32), ("stop", C.POINTER(DegStopModel)), ("trace", C.c_void_p),
                ("trace_rows_per_query", C.c_int64), ("trace_interval", C.c_int32),
                ("waves_per_cu", C.c_int32), ("queue_lds", C.c_int32),
                ("exclude_offsets", C.c_void_p), ("exclude_ids", C.c_void_p)]


class DegQueryDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("seed_or_vertex", C.c_int32), ("query_row", C.c_int64),
                ("k", C.c_int32), ("eps", C.c_float), ("out_offset", C.c_int64)]


class DegBuildParams(C.Structure):
    _fields_ = [("degree", C.c_int32), ("k_ext", C.c_int32), ("eps_ext", C.c_float),
                ("lag", C.c_int32), ("batch", C.c_int64)]


EXPORTS = [
    "deg_search_workspace_bytes", "deg_search_resident_waves", "deg_search", "deg_search_noalloc",
    "deg_search_indexed",
    "deg_search_batch", "deg_build_graph", "deg_graph_check_mrng",
    "deg_knn_workspace_bytes", "deg_knn_bruteforce", "deg_medoid_workspace_bytes", "deg_medoid",
    "deg_encode_bf16", "deg_encode_fp8", "deg_mlp_workspace_bytes", "deg_mlp_train_step",
    "deg_mlp_forward", "deg_mlp_forward_bf16", "deg_mlp_export_bf16", "deg_mlp_feature_stats",
    "deg_mlp_standardise", "deg_tune_register",
    "deg_tune_clear", "deg_device_cu_count", "deg_status_string",
]

_lib = None


def load_library(path: Path | None = None):
    """Loads libdeg.so (no GPU needed to load). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    p = Path(path or LIB_PATH)
    if not p.exists():
        raise RuntimeError("libdeg.so is not built: run `python -m paper_2307_10479_amd.build_lib`")
    L = C.CDLL(str(p))
    V, P, I32, I64, F, SZ = C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
    pv, pg, po = C.POINTER(DegVectors), C.POINTER(DegGraph), C.POINTER(DegSearchOpts)
    sigs = {
        "deg_search_workspace_bytes": (SZ, [pv, pg, I64, I32, po]),
        "deg_search_resident_waves": (I32, [pv, pg, I32, po]),
        "deg_build_graph": (I32, [pv, P, I64, C.POINTER(DegBuildParams), P, P, P, V]),
        "deg_graph_check_mrng": (I32, [pg, P, I64, P, P, P, V]),
        "deg_search": (I32, [pv, pg, P, I64, I64, P, I32, I32, F, po, P, P, P, P, SZ, V]),
        "deg_search_noalloc": (I32, [pv, pg, P, I64, I64, P, I32, I32, F, po, P, P, P, V]),
        "deg_search_indexed": (I32, [pv, pg, P, I64, I32, F, po, P, P, P, P, SZ, V]),
        "deg_search_batch": (I32, [pv, pg, P, I64, I64, P, I64, I32, po, P, P, P, P, SZ, V]),
        "deg_knn_workspace_bytes": (SZ, [I64, I32, I64, I32]),
        "deg_knn_bruteforce": (I32, [P, I64, I32, I64, P, I64, I64, I32, I32, P, P, P, P, SZ, V]),
        "deg_medoid_workspace_bytes": (SZ, [I64, I32]),
        "deg_medoid": (I32, [P, I64, I32, I64, I32, P, P, SZ, V]),
        "deg_encode_bf16": (I32, [P, I64, I32, I64, P, I64, V]),
        "deg_encode_fp8": (I32, [P, I64, I32, I64, P, I64, P, V]),
        "deg_mlp_workspace_bytes": (SZ, [I64]),
        "deg_mlp_train_step": (I32, [P, P, P, P, P, I64, I64, F, P, P, P, SZ, V]),
        "deg_mlp_forward": (I32, [P, P, I64, P, V]),
        "deg_mlp_forward_bf16": (I32, [P, P, I64, P, V]),
        "deg_mlp_export_bf16": (I32, [P, P, V]),
        "deg_mlp_feature_stats": (I32, [P, I64, P, P, V]),
        "deg_mlp_standardise": (I32, [P, I64, P, P, P, V]),
        "deg_tune_register": (I32, [I32, I32, I32, I32, I32, I32]),
        "deg_tune_clear": (None, []),
        "deg_device_cu_count": (I32, []),
        "deg_status_string": (C.c_char_p, [I32]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def lib():
    L = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("the DEG library needs a ROCm GPU; none is visible")
    return L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(fn, code):
    if code != 0:
        raise DegError(fn, code)


_ws_cache: dict = {}
_ws_retired: list = []


def workspace(nbytes: int, tag: str = "search") -> torch.Tensor:
    """A cached device workspace of at least nbytes for the current stream.

    One buffer per (tag, stream), so that calls on different streams never
    share the work counter or the visited tables. A buffer that is outgrown is
    kept alive (not freed), so that a HIP graph captured with it stays valid;
    release_workspaces() drops them all. Callers that capture graphs can also
    pass their own buffer (the `workspace=` argument of the search calls)."""
    key = (tag, torch.cuda.current_stream().cuda_stream)
    t = _ws_cache.get(key)
    if t is None or t.numel() < nbytes:
        if t is not None:
            _ws_retired.append(t)
        t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
        _ws_cache[key] = t
    return t


def release_workspaces() -> None:
    """Frees every cached workspace (no captured graph may use them afterwards)."""
    _ws_cache.clear()
    _ws_retired.clear()


def _ws_arg(given, need: int, tag: str = "search") -> torch.Tensor:
    if given is None:
        return workspace(need, tag)
    if not (given.is_cuda and given.dtype == torch.uint8) or given.numel() < need:
        raise DegError("workspace", 3)
    return given


def _pad4(x: int) -> int:
    return (x + 3) // 4 * 4


# ------------------------------------------------------------------ stores
class VectorStore:
    """Base vectors on the device: FP32 rows plus the traversal store.

    dtype 'f32' traverses the FP32 rows; 'bf16' and 'fp8' build a second store
    with the library's encoders (round to nearest even; FP8 with one scale per
    row) and keep the FP32 rows for the exact rerank.
    """

    def __init__(self, base: torch.Tensor, dtype: str = "f32", metric: int = L2):
        L = lib()
        assert base.is_cuda and base.dtype == torch.float32 and base.dim() == 2
        n, m = base.shape
        self.n, self.dim, self.metric, self.dtype_name = n, m, metric, dtype
        self.dtype = DTYPES[dtype]
        stride = _pad4(m)
        if base.stride(0) == stride and base.is_contiguous():
            f32 = base
        else:
            f32 = torch.zeros((n, stride), dtype=torch.float32, device=base.device)
            f32[:, :m] = base
        self.f32 = f32
        self.f32_stride = stride
        self.scale = None
        if self.dtype == F32:
            self.data, self.stride = f32, stride
        elif self.dtype == BF16:
            self.data = torch.empty((n, stride), dtype=torch.uint16, device=base.device)
            _check("deg_encode_bf16", L.deg_encode_bf16(_ptr(f32), n, m, stride, _ptr(self.data),
                                                        stride, _stream()))
            self.stride = stride
        else:
            self.data = torch.empty((n, stride), dtype=torch.uint8, device=base.device)
            self.scale = torch.empty(n, dtype=torch.float32, device=base.device)
            _check("deg_encode_fp8", L.deg_encode_fp8(_ptr(f32), n, m, stride, _ptr(self.data),
                                                      stride, _ptr(self.scale), _stream()))
            self.stride = stride

    def c(self) -> DegVectors:
        return DegVectors(self.data.data_ptr(), self.n, self.dim, self.stride, self.dtype,
                          self.metric, None if self.scale is None else self.scale.data_ptr(),
                          self.f32.data_ptr(), self.f32_stride, 0)

    def row_bytes(self) -> int:
        """Bytes of one traversal row as the search reads it."""
        return {F32: 4 * self.dim, BF16: 2 * self.dim, FP8: self.dim + 4}[self.dtype]


class DeviceGraph:
    """Adjacency on the device. Rows are padded (with -1, never read) to a
    multiple of `row_align` ids, so that with 30 neighbours a row is one
    128-byte line instead of straddling two; row_align=1 keeps the given layout."""

    def __init__(self, adj: torch.Tensor, row_align: int = 32):
        assert adj.is_cuda and adj.dtype == torch.int32 and adj.dim() == 2 and adj.is_contiguous()
        self.n, self.degree = adj.shape
        stride = -(-self.degree // row_align) * row_align
        if stride != self.degree:
            padded = torch.full((self.n, stride), -1, dtype=torch.int32, device=adj.device)
            padded[:, :self.degree] = adj
            adj = padded
        self.adj = adj
        self.stride = stride

    def c(self) -> DegGraph:
        return DegGraph(self.adj.data_ptr(), self.n, self.degree, self.stride)


class StopModel:
    """BF16 stop-predictor weights plus feature standardisation, on the device."""

    def __init__(self, weights_bf16: torch.Tensor, mean: torch.Tensor, inv_std: torch.Tensor,
                 tau: float, interval: int, tau_long: float | None = None, long_hops: int = 0):
        self.w, self.mean, self.inv_std = weights_bf16, mean, inv_std
        self.tau, self.interval = float(tau), int(interval)
        self.tau_long = float(tau if tau_long is None else tau_long)
        self.long_hops = int(long_hops)

    def c(self) -> DegStopModel:
        return DegStopModel(self.w.data_ptr(), self.mean.data_ptr(), self.inv_std.data_ptr(),
                            self.tau, self.interval, self.tau_long, self.long_hops)


def _opts(queue_cap=0, hash_slots=0, k_pool=0, rerank=False, stop: StopModel | None = None,
          trace=None, trace_rows=0, trace_interval=0, waves_per_cu=0, queue_lds=0, exclude=None):
    o = DegSearchOpts()
    o.queue_cap, o.hash_slots, o.k_pool, o.rerank = int(queue_cap), int(hash_slots), int(k_pool), int(bool(rerank))
    keep = None
    if stop is not None:
        keep = stop.c()
        o.stop = C.pointer(keep)
    if trace is not None:
        o.trace = trace.data_ptr()
        o.trace_rows_per_query = int(trace_rows)
        o.trace_interval = int(trace_interval)
    o.waves_per_cu = int(waves_per_cu)
    o.queue_lds = int(queue_lds)
    if exclude is not None:  # (offsets int64 [nq + 1], ids int32) device tensors
        o.exclude_offsets = exclude[0].data_ptr()
        o.exclude_ids = exclude[1].data_ptr()
    return o, keep


def exclusion_lists(lists) -> tuple:
    """Device CSR form of per-query exclusion lists (a sequence of id sequences)."""
    import numpy as np
    off = np.zeros(len(lists) + 1, np.int64)
    off[1:] = np.cumsum([len(x) for x in lists])
    ids = np.array([v for x in lists for v in x] or [0], np.int32)
    return torch.from_numpy(off).cuda(), torch.from_numpy(ids).cuda()


# ------------------------------------------------------------------ search
def search_workspace_bytes(store, graph, nq, k, **opts) -> int:
    o, _keep = _opts(**opts)
    v, g = store.c(), graph.c()
    return int(lib().deg_search_workspace_bytes(C.byref(v), C.byref(g), nq, k, C.byref(o)))


def resident_waves_per_cu(store, graph, k, k_pool=0, hash_slots=0, **opts) -> int:
    """Waves per CU a search launch with these options keeps resident."""
    o, _keep = _opts(k_pool=k_pool, hash_slots=hash_slots, **opts)
    v, g = store.c(), graph.c()
    return int(lib().deg_search_resident_waves(C.byref(v), C.byref(g), k, C.byref(o)))


def search(store: VectorStore, graph: DeviceGraph, queries: torch.Tensor, seeds: torch.Tensor,
           k: int, eps: float, out=None, workspace=None, **opts):
    """RangeSearch (Algorithm 1) of every query row. Returns (ids, dists, stats)."""
    L = lib()
    assert queries.is_cuda and queries.dtype == torch.float32 and queries.dim() == 2
    assert queries.stride(1) == 1
    nq = queries.shape[0]
    if seeds.dim() == 1:
        seeds = seeds.view(-1, 1).expand(nq, seeds.numel()) if seeds.numel() != nq else seeds.view(-1, 1)
    seeds = seeds.to(device=queries.device, dtype=torch.int32).contiguous()
    o, _keep = _opts(**opts)
    v, g = store.c(), graph.c()
    if out is None:
        ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
        ds = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
        st = torch.empty((nq, 4), dtype=torch.int32, device=queries.device)
    else:
        ids, ds, st = out
    need = L.deg_search_workspace_bytes(C.byref(v), C.byref(g), nq, k, C.byref(o))
    ws = _ws_arg(workspace, need)
    _check("deg_search", L.deg_search(C.byref(v), C.byref(g), _ptr(queries), nq, queries.stride(0),
                                      _ptr(seeds), seeds.shape[1], k, float(eps), C.byref(o),
                                      _ptr(ids), _ptr(ds), _ptr(st), _ptr(ws), ws.numel(),
                                      _stream()))
    return ids, ds, st


def search_noalloc(store: VectorStore, graph: DeviceGraph, queries: torch.Tensor,
                   seeds: torch.Tensor, k: int, eps: float, out=None, **opts):
    """search() through deg_search_noalloc: no workspace (the library's own
    per-GPU scratch array). Outputs are allocated here unless `out` is given."""
    L = lib()
    assert queries.is_cuda and queries.dtype == torch.float32 and queries.dim() == 2
    assert queries.stride(1) == 1
    nq = queries.shape[0]
    if seeds.dim() == 1:
        seeds = seeds.view(-1, 1).expand(nq, seeds.numel()) if seeds.numel() != nq else seeds.view(-1, 1)
    seeds = seeds.to(device=queries.device, dtype=torch.int32).contiguous()
    o, _keep = _opts(**opts)
    v, g = store.c(), graph.c()
    if out is None:
        ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
        ds = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
        st = torch.empty((nq, 4), dtype=torch.int32, device=queries.device)
    else:
        ids, ds, st = out
    _check("deg_search_noalloc", L.deg_search_noalloc(C.byref(v), C.byref(g), _ptr(queries), nq,
                                                      queries.stride(0), _ptr(seeds),
                                                      seeds.shape[1], k, float(eps), C.byref(o),
                                                      _ptr(ids), _ptr(ds), _ptr(st), _stream()))
    return ids, ds, st


def search_indexed(store: VectorStore, graph: DeviceGraph, qids: torch.Tensor, k: int, eps: float,
                   out=None, workspace=None, **opts):
    """Exploratory search: each query is a base vertex, excluded from its answer."""
    L = lib()
    qids = qids.to(device="cuda", dtype=torch.int32).contiguous()
    nq = qids.numel()
    o, _keep = _opts(**opts)
    v, g = store.c(), graph.c()
    if out is None:
        ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
        ds = torch.empty((nq, k), dtype=torch.float32, device="cuda")
        st = torch.empty((nq, 4), dtype=torch.int32, device="cuda")
    else:
        ids, ds, st = out
    need = L.deg_search_workspace_bytes(C.byref(v), C.byref(g), nq, k, C.byref(o))
    ws = _ws_arg(workspace, need)
    _check("deg_search_indexed", L.deg_search_indexed(C.byref(v), C.byref(g), _ptr(qids), nq, k,
                                                      float(eps), C.byref(o), _ptr(ids), _ptr(ds),
                                                      _ptr(st), _ptr(ws), ws.numel(), _stream()))
    return ids, ds, st


def make_descs(kind, seed_or_vertex, query_row, k, eps) -> tuple[torch.Tensor, int, int]:
    """Packs per-query descriptors (numpy/torch arrays) into a device buffer.

    Results of query i start at out_offset = sum of the k of the queries before it.
    Returns (device bytes, total result slots, k_max).
    """
    import numpy as np
    kind = np.asarray(kind, np.int32)
    nq = kind.shape[0]
    arr = (DegQueryDesc * nq)()
    kk = np.asarray(k, np.int64)
    offs = np.concatenate([[0], np.cumsum(kk)[:-1]]).astype(np.int64)
    sv = np.asarray(seed_or_vertex, np.int64)
    qr = np.asarray(query_row, np.int64)
    ee = np.asarray(eps, np.float32)
    buf = np.zeros(nq, dtype=np.dtype([("kind", "<i4"), ("sv", "<i4"), ("row", "<i8"),
                                       ("k", "<i4"), ("eps", "<f4"), ("off", "<i8")]))
    assert buf.itemsize == C.sizeof(DegQueryDesc)
    buf["kind"], buf["sv"], buf["row"], buf["k"], buf["eps"], buf["off"] = kind, sv, qr, kk, ee, offs
    del arr
    dev = torch.from_numpy(buf.view(np.uint8).copy()).cuda()
    return dev, int(kk.sum()), int(kk.max()) if nq else 1


def search_batch(store: VectorStore, graph: DeviceGraph, queries: torch.Tensor | None,
                 descs: torch.Tensor, nq: int, total: int, k_max: int, workspace=None, **opts):
    """Mixed stream in one persistent launch. Returns flat ids/dists (total) and stats (nq x 4)."""
    L = lib()
    o, _keep = _opts(**opts)
    v, g = store.c(), graph.c()
    ids = torch.empty(total, dtype=torch.int32, device="cuda")
    ds = torch.empty(total, dtype=torch.float32, device="cuda")
    st = torch.empty((nq, 4), dtype=torch.int32, device="cuda")
    need = L.deg_search_workspace_bytes(C.byref(v), C.byref(g), nq, k_max, C.byref(o))
    ws = _ws_arg(workspace, need)
    qs = 0 if queries is None else queries.stride(0)
    nrows = 0 if queries is None else queries.shape[0]
    _check("deg_search_batch", L.deg_search_batch(C.byref(v), C.byref(g), _ptr(queries), nrows, qs,
                                                  _ptr(descs), nq, k_max, C.byref(o), _ptr(ids),
                                                  _ptr(ds), _ptr(st), _ptr(ws), ws.numel(),
                                                  _stream()))
    return ids, ds, st


# ------------------------------------------------------------------ ground truth, seed
def knn_bruteforce(base: torch.Tensor, queries: torch.Tensor, k: int, metric: int = L2,
                   exclude: torch.Tensor | None = None):
    L = lib()
    n, m = base.shape
    nq = queries.shape[0]
    if base.stride(0) % 4 or base.stride(1) != 1:  # rows are read as float4: pad to 4 columns
        padded = torch.zeros((n, _pad4(m)), dtype=torch.float32, device=base.device)
        padded[:, :m] = base
        base = padded
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    ds = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    ex = None if exclude is None else exclude.to(device="cuda", dtype=torch.int32).contiguous()
    ws = workspace(L.deg_knn_workspace_bytes(n, m, nq, k), "knn")
    _check("deg_knn_bruteforce", L.deg_knn_bruteforce(_ptr(base), n, m, base.stride(0),
                                                      _ptr(queries), nq, queries.stride(0), k,
                                                      metric, _ptr(ex), _ptr(ids), _ptr(ds),
                                                      _ptr(ws), ws.numel(), _stream()))
    return ids, ds


def medoid(base: torch.Tensor, metric: int = L2) -> int:
    L = lib()
    n, m = base.shape
    out = torch.empty(1, dtype=torch.int32, device="cuda")
    ws = workspace(L.deg_medoid_workspace_bytes(n, m), "medoid")
    _check("deg_medoid", L.deg_medoid(_ptr(base), n, m, base.stride(0), metric, _ptr(out),
                                      _ptr(ws), ws.numel(), _stream()))
    return int(out.item())


# ------------------------------------------------------------------ construction
def build_graph(store: VectorStore, host_base, degree, k_ext, eps_ext, batch=4096, lag=0):
    """Graph construction (Sec. 5.2, Algorithm 3 without optimizeEdge) with the
    searches of each block of new vertices batched on the GPU.

    store: the FP32 VectorStore of all n vectors; host_base: the same (n, dim)
    float32 array on the host. Returns (adjacency (n, degree) int32 on the device,
    weights (n, degree) float32 numpy, counters dict)."""
    import numpy as np
    hb = np.ascontiguousarray(host_base, dtype=np.float32)
    n = store.n
    if hb.shape[0] != n or hb.shape[1] != store.dim:
        raise ValueError("host_base must be the store's %d x %d vectors" % (n, store.dim))
    adj = torch.empty((n, degree), dtype=torch.int32, device="cuda")
    w = np.empty((n, degree), np.float32)
    cnt = np.zeros(6, np.int64)
    p = DegBuildParams(degree=int(degree), k_ext=int(k_ext), eps_ext=float(eps_ext), lag=int(lag),
                       batch=int(batch))
    v = store.c()
    _check("deg_build_graph", lib().deg_build_graph(
        C.byref(v), C.c_void_p(hb.ctypes.data), hb.shape[1], C.byref(p), _ptr(adj),
        C.c_void_p(w.ctypes.data), C.c_void_p(cnt.ctypes.data), _stream()))
    return adj, w, dict(zip(["blocks", "searches", "phase2", "lossy", "search_us", "edit_us"],
                            cnt.tolist()))


def check_mrng(graph: DeviceGraph, weights: torch.Tensor):
    """MRNG conformity of every edge (Algorithm 2) and every vertex's longest edge.
    weights: (n, >= degree) FP32 on the device, row-aligned with the adjacency.
    Returns (ok (n, degree) uint8 on the device: 1 passes, 0 fails, 255 empty slot;
    number of failing entries; slot of each vertex's longest edge (n,) int32)."""
    n, d = graph.n, graph.degree
    if not (weights.is_cuda and weights.dtype == torch.float32 and weights.dim() == 2
            and weights.shape[0] == n and weights.shape[1] >= d and weights.stride(1) == 1):
        raise ValueError("weights must be a (n, >= degree) float32 device tensor")
    ok = torch.empty((n, d), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    longest = torch.empty(n, dtype=torch.int32, device="cuda")
    g = graph.c()
    _check("deg_graph_check_mrng", lib().deg_graph_check_mrng(
        C.byref(g), _ptr(weights), weights.stride(0), _ptr(ok), _ptr(cnt), _ptr(longest),
        _stream()))
    return ok, cnt, longest


# ------------------------------------------------------------------ MLP
def mlp_train_step(params, m, v, X, y, step, lr, grad=None, loss=None):
    L = lib()
    B = X.shape[0]
    ws = workspace(L.deg_mlp_workspace_bytes(B), "mlp")
    _check("deg_mlp_train_step", L.deg_mlp_train_step(_ptr(params), _ptr(m), _ptr(v), _ptr(X),
                                                      _ptr(y), B, int(step), float(lr), _ptr(grad),
                                                      _ptr(loss), _ptr(ws), ws.numel(), _stream()))


def mlp_forward(params, X):
    out = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
    _check("deg_mlp_forward", lib().deg_mlp_forward(_ptr(params), _ptr(X), X.shape[0], _ptr(out),
                                                    _stream()))
    return out


def mlp_forward_bf16(w, X):
    out = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
    _check("deg_mlp_forward_bf16", lib().deg_mlp_forward_bf16(_ptr(w), _ptr(X), X.shape[0],
                                                              _ptr(out), _stream()))
    return out


def mlp_export_bf16(params):
    out = torch.empty(MLP_NPARAMS, dtype=torch.uint16, device="cuda")
    _check("deg_mlp_export_bf16", lib().deg_mlp_export_bf16(_ptr(params), _ptr(out), _stream()))
    return out


def mlp_feature_stats(X):
    """Per-feature mean and inverse standard deviation of B x 16 rows (library kernel)."""
    mean = torch.empty(NFEAT, dtype=torch.float32, device="cuda")
    inv = torch.empty(NFEAT, dtype=torch.float32, device="cuda")
    _check("deg_mlp_feature_stats", lib().deg_mlp_feature_stats(_ptr(X), X.shape[0], _ptr(mean),
                                                                _ptr(inv), _stream()))
    return mean, inv


def mlp_standardise(X, mean, inv_std):
    out = torch.empty_like(X)
    _check("deg_mlp_standardise", lib().deg_mlp_standardise(_ptr(X), X.shape[0], _ptr(mean),
                                                            _ptr(inv_std), _ptr(out), _stream()))
    return out


def tune_register(dtype, dim, degree, kp_bucket, hash_slots, waves_per_cu):
    _check("deg_tune_register", lib().deg_tune_register(dtype, dim, degree, kp_bucket, hash_slots,
                                                        waves_per_cu))


def tune_clear():
    lib().deg_tune_clear()


def cu_count() -> int:
    return int(lib().deg_device_cu_count())
