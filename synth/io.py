"""Graph file format shared by the build script, the tests and the benchmark.

Layout: 4-byte magic b"DEGG", then int32 version, int64 n, int32 d, int32
metric (0 = L2, 1 = IP), int32 has_weights, int32 reserved (32 bytes in all).
Version 1 then holds int32 adjacency n x d and (if has_weights) float32
weights n x d. Version 2 holds every row's neighbours in ascending id order,
each row as its first id followed by the differences to the previous id, as
int32 split into its four byte planes (all low bytes, then all second bytes,
...) and zlib-compressed (a uint64 byte count first), then (if has_weights)
the weights permuted alongside, float32, uncompressed. A row's order does not
matter to the search (a hop expands its whole row at once and every ordering
is by (distance, id)). This module only reads and writes bytes.
"""
from __future__ import annotations

import os
import zlib

import numpy as np

MAGIC = b"DEGG"


def _header(version, n, d, metric, has_w):
    hdr = np.zeros(7, np.int32)
    hdr[0] = version
    hdr[1:3] = np.array([n], np.int64).view(np.int32)
    hdr[3] = d
    hdr[4] = metric
    hdr[5] = has_w
    return hdr


def save_graph(path, adj, metric=0, w=None, compact=True):
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    n, d = adj.shape
    tmp = str(path) + ".tmp"
    with open(tmp, "wb") as f:
        f.write(MAGIC)
        if compact:
            f.write(_header(2, n, d, metric, 0 if w is None else 1).tobytes())
            order = np.argsort(adj, axis=1, kind="stable")
            rows = np.take_along_axis(adj, order, axis=1)
            delta = np.diff(rows, axis=1, prepend=0).astype(np.int32)
            planes = np.ascontiguousarray(delta.reshape(-1).view(np.uint8).reshape(-1, 4).T)
            blob = zlib.compress(planes.tobytes(), 6)
            f.write(np.array([len(blob)], np.uint64).tobytes())
            f.write(blob)
            if w is not None:
                ws = np.take_along_axis(np.asarray(w, np.float32), order, axis=1)
                f.write(np.ascontiguousarray(ws, dtype=np.float32).tobytes())
        else:
            f.write(_header(1, n, d, metric, 0 if w is None else 1).tobytes())
            f.write(adj.tobytes())
            if w is not None:
                f.write(np.ascontiguousarray(w, dtype=np.float32).tobytes())
    os.replace(tmp, path)


def load_graph(path, with_weights=False):
    """Returns (adj int32 n x d, metric, weights or None)."""
    with open(path, "rb") as f:
        if f.read(4) != MAGIC:
            raise ValueError("%s: not a DEG graph file" % path)
        hdr = np.frombuffer(f.read(28), np.int32)
        version = int(hdr[0])
        n = int(hdr[1:3].view(np.int64)[0])
        d, metric, has_w = int(hdr[3]), int(hdr[4]), int(hdr[5])
        if version == 1:
            adj = np.fromfile(f, dtype=np.int32, count=n * d).reshape(n, d)
        elif version == 2:
            size = int(np.frombuffer(f.read(8), np.uint64)[0])
            planes = np.frombuffer(zlib.decompress(f.read(size)), np.uint8).reshape(4, n * d)
            delta = np.ascontiguousarray(planes.T).view(np.int32).reshape(n, d)
            adj = np.cumsum(delta, axis=1, dtype=np.int64).astype(np.int32)
        else:
            raise ValueError("%s: unknown graph file version %d" % (path, version))
        w = None
        if has_w and with_weights:
            w = np.fromfile(f, dtype=np.float32, count=n * d).reshape(n, d)
    return adj, metric, w
