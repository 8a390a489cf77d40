"""Graph file format shared by the build script, the tests and the benchmark.

Layout: 4-byte magic b"DEGG", then int32 version (1), int64 n, int32 d,
int32 metric (0 = L2, 1 = IP), int32 has_weights, int32 reserved (32 bytes in
all), then int32 adjacency n x d, then (if has_weights) float32 weights n x d.
This module only reads and writes bytes.
"""
from __future__ import annotations

import os

import numpy as np

MAGIC = b"DEGG"


def save_graph(path, adj, metric=0, w=None):
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    n, d = adj.shape
    hdr = np.zeros(7, np.int32)
    hdr[0] = 1
    hdr[1:3] = np.array([n], np.int64).view(np.int32)
    hdr[3] = d
    hdr[4] = metric
    hdr[5] = 0 if w is None else 1
    tmp = str(path) + ".tmp"
    with open(tmp, "wb") as f:
        f.write(MAGIC)
        f.write(hdr.tobytes())
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
        n = int(hdr[1:3].view(np.int64)[0])
        d, metric, has_w = int(hdr[3]), int(hdr[4]), int(hdr[5])
        adj = np.fromfile(f, dtype=np.int32, count=n * d).reshape(n, d)
        w = None
        if has_w and with_weights:
            w = np.fromfile(f, dtype=np.float32, count=n * d).reshape(n, d)
    return adj, metric, w
