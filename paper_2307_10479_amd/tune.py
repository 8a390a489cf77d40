"""Autotuner for the persistent search launch.

For one (store dtype, dim, degree, pool-size bucket) it times the search on a
sample of queries over a grid of LDS visited-table sizes and resident waves
per CU, keeps the fastest, and registers it with the library
(deg_tune_register), which every later launch of that shape uses. Neither
knob changes results: the visited set is exact whether it stays in LDS or
spills to the workspace, and the grid size only changes how many queries are
in flight. Results are cached in a JSON file keyed by the device name.
"""
from __future__ import annotations

import json
import os
from pathlib import Path

import torch

from . import api

CACHE = Path(os.environ.get("DEG_TUNE_CACHE", Path.home() / ".cache" / "deg_tune.json"))
HASH_SLOTS = (256, 512, 1024, 2048, 4096, 8192)
WAVES_PER_CU = (0, 4, 6, 8, 12, 16)


def _key(dtype, dim, degree, bucket):
    return "%s|%d|%d|%d|%d" % (torch.cuda.get_device_name(0), dtype, dim, degree, bucket)


def kp_bucket(kp: int) -> int:
    return 16 if kp <= 16 else 64 if kp <= 64 else 128 if kp <= 128 else 256 if kp <= 256 else 512


def load_cache() -> dict:
    try:
        return json.loads(CACHE.read_text())
    except Exception:
        return {}


def apply_cache(cache: dict | None = None) -> int:
    """Registers every cached entry for this device; returns how many."""
    cache = load_cache() if cache is None else cache
    dev = torch.cuda.get_device_name(0)
    n = 0
    for key, e in cache.items():
        name, dtype, dim, degree, bucket = key.split("|")
        if name != dev:
            continue
        api.tune_register(int(dtype), int(dim), int(degree), int(bucket), e["hash_slots"],
                          e["waves_per_cu"])
        n += 1
    return n


def _time(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(store, graph, queries, seeds, k, eps, k_pool=0, save=True, **opts):
    """Times the grid on (queries, seeds) and registers the fastest setting."""
    kp = max(k, k_pool)
    table = []
    for hs in HASH_SLOTS:
        for w in WAVES_PER_CU:
            try:
                ms = _time(lambda: api.search(store, graph, queries, seeds, k, eps, k_pool=k_pool,
                                              hash_slots=hs, waves_per_cu=w, **opts))
            except api.DegError:
                continue
            table.append(dict(hash_slots=hs, waves_per_cu=w, ms=ms))
    # the library caps a request at the resident waves; record the effective value
    # (0 = all resident) so that a cached setting never claims more than ran
    for r in table:
        if r["waves_per_cu"] and api.resident_waves_per_cu(store, graph, k, k_pool, r["hash_slots"],
                                                         **opts) <= r["waves_per_cu"]:
            r["waves_per_cu"] = 0
    best = min(table, key=lambda r: r["ms"])
    bucket = kp_bucket(kp)
    api.tune_register(store.dtype, store.dim, graph.degree, bucket, best["hash_slots"],
                      best["waves_per_cu"])
    if save:
        cache = load_cache()
        cache[_key(store.dtype, store.dim, graph.degree, bucket)] = dict(
            hash_slots=best["hash_slots"], waves_per_cu=best["waves_per_cu"], ms=best["ms"])
        try:
            CACHE.parent.mkdir(parents=True, exist_ok=True)
            CACHE.write_text(json.dumps(cache, indent=1))
        except OSError:
            pass
    return best, table
