"""Learned early stop for the range search: trace -> train -> calibrate.

1. Traces: the plain search runs with tracing on; every `interval` hops it
   writes its 16 state features (hop and evaluation counts, best/k-th and
   radius ratios, stagnation counters, acceptance fractions, the share of
   queued candidates closer than the k-th result, the popped distance over
   the k-th distance, eps, k, exploratory flag, visited count). At the end of a query each row
   is labelled 1 when the top-10 results no longer change afterwards.
2. Training: the 16-64-64-1 MLP is trained with the library's FP32 forward /
   backward / Adam kernels on standardised features (mean binary
   cross-entropy).
3. Calibration: on held-out queries the threshold tau is the smallest value
   whose top-10 agreement with the plain search stays >= 1 - max_loss; the
   plain stopping rule remains the fallback.
The torch calls here only move, select and batch data; all arithmetic of the
search, the feature statistics and standardisation, the network and its
training runs in libdeg.so.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


def collect_traces(store, graph, queries, seeds, k, eps_values, interval=2, rows=64,
                   chunk=50_000, **opts):
    """Runs the plain search with tracing; returns (X, y) on the device (rows with a label)."""
    Xs, ys = [], []
    nq = queries.shape[0]
    per = (nq + len(eps_values) - 1) // len(eps_values)
    for ei, eps in enumerate(eps_values):
        lo, hi = ei * per, min(nq, (ei + 1) * per)
        for s in range(lo, hi, chunk):
            e = min(hi, s + chunk)
            n = e - s
            trace = torch.empty(n * rows * api.TRACE_W, dtype=torch.float32, device="cuda")
            api.search(store, graph, queries[s:e], seeds[s:e], k, float(eps), trace=trace,
                       trace_rows=rows, trace_interval=interval, **opts)
            T = trace.view(n * rows, api.TRACE_W)
            keep = T[:, 16] >= 0
            Xs.append(T[keep, :16].clone())
            ys.append(T[keep, 16].clone())
            del trace, T
    return torch.cat(Xs), torch.cat(ys)


def standardise(X):
    """Feature means and inverse standard deviations (library kernel)."""
    return api.mlp_feature_stats(X.contiguous())


def standardised(X, mean, inv_std):
    """(X - mean) * inv_std in FP32 (library kernel), the rounding the search applies."""
    return api.mlp_standardise(X.contiguous(), mean, inv_std)


def train(X, y, epochs=4, batch=8192, lr=2e-3, seed=0):
    """Trains the MLP with the library's kernels. Returns FP32 params and the loss history."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    params = torch.empty(api.MLP_NPARAMS, dtype=torch.float32)
    # He-style init: W1 (64x16), b1, W2 (64x64), b2, w3 (64), b3
    params[:1024] = torch.randn(1024, generator=g) * (2.0 / 16) ** 0.5
    params[1024:1088] = 0.0
    params[1088:5184] = torch.randn(4096, generator=g) * (2.0 / 64) ** 0.5
    params[5184:5248] = 0.0
    params[5248:5312] = torch.randn(64, generator=g) * (1.0 / 64) ** 0.5
    params[5312] = 0.0
    params = params.cuda()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    n = X.shape[0]
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).cuda()
        tot = 0.0
        nb = 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            xb = X[idx].contiguous()
            yb = y[idx].contiguous()
            step += 1
            api.mlp_train_step(params, m, v, xb, yb, step, lr, loss=loss)
            if nb % 64 == 0:
                tot += loss.item()
            nb += 1
        hist.append(tot / max(1, (nb + 63) // 64))
    return params, hist


def build_model(params, mean, inv_std, tau, interval, tau_long=None, long_hops=0):
    w = api.mlp_export_bf16(params)
    return api.StopModel(w, mean, inv_std, tau, interval, tau_long, long_hops)


def build_model_from_bf16(w, mean, inv_std, tau, interval, tau_long=None, long_hops=0):
    return api.StopModel(w, mean, inv_std, tau, interval, tau_long, long_hops)


def calibrate_long(run, run_plain_ids, agree_fn, params, mean, inv_std, tau, interval,
                   max_loss=0.005, long_hops=(1024, 2048, 3072),
                   taus_long=(0.5, 0.6, 0.7, 0.8, 0.9), reps=2):
    """Second threshold for long queries: among (long_hops, tau_long <= tau) whose
    agreement with the plain search stays >= 1 - max_loss, the fastest on the
    held-out queries (timed; `run(model)` launches the search, returns ids first).
    Returns (tau_long, long_hops, table); (tau, 0) when none is faster."""
    def timed(model):
        run(model)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            out = run(model)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out
    base_ms, _ = timed(build_model(params, mean, inv_std, tau, interval))
    best = (tau, 0, base_ms)
    table = [(0, tau, 1.0, base_ms)]
    for lh in long_hops:
        for tl in taus_long:
            if tl >= tau:
                continue
            ms, out = timed(build_model(params, mean, inv_std, tau, interval, tl, lh))
            agree = agree_fn(out[0], run_plain_ids)
            table.append((lh, tl, agree, ms))
            if agree >= 1.0 - max_loss and ms < best[2]:
                best = (tl, lh, ms)
    return best[0], best[1], table


def top10_agreement(a_ids, b_ids, k=10):
    a = a_ids[:, :k].cpu().numpy()
    b = b_ids[:, :k].cpu().numpy()
    hit = 0
    for x, z in zip(a, b):
        hit += len(set(x.tolist()) & set(z.tolist()))
    return hit / (k * a.shape[0])


def calibrate(store, graph, queries, seeds, k, eps, params, mean, inv_std, interval,
              max_loss=0.005, taus=(0.5, 0.6, 0.7, 0.8, 0.85, 0.9, 0.93, 0.95, 0.97, 0.98, 0.99, 0.995),
              **opts):
    """Smallest tau whose top-10 agreement with the plain search is >= 1 - max_loss."""
    plain = api.search(store, graph, queries, seeds, k, eps, **opts)
    best = None
    table = []
    for tau in taus:
        model = build_model(params, mean, inv_std, tau, interval)
        got = api.search(store, graph, queries, seeds, k, eps, stop=model, **opts)
        agree = top10_agreement(got[0], plain[0], min(10, k))
        hops = float(got[2][:, 0].float().mean())
        table.append((tau, agree, hops))
        if best is None and agree >= 1.0 - max_loss:
            best = tau
    return (best if best is not None else 1.0), table


def traces_from(run, n, rows, interval):
    """Trace rows of one plain search over n queries: `run(**trace_opts)` launches it.
    Returns (X, y) on the device (rows that received a label)."""
    trace = torch.empty(n * rows * api.TRACE_W, dtype=torch.float32, device="cuda")
    run(trace=trace, trace_rows=rows, trace_interval=interval)
    T = trace.view(n * rows, api.TRACE_W)
    keep = T[:, 16] >= 0
    return T[keep, :16].clone(), T[keep, 16].clone()


def agreement_flat(a_ids, b_ids, ks, offsets):
    """Mean top-min(10, k) agreement of two flat result buffers (one k per query)."""
    a = a_ids.cpu().numpy()
    b = b_ids.cpu().numpy()
    tot = 0.0
    for k, o in zip(np.asarray(ks).tolist(), np.asarray(offsets).tolist()):
        t = min(10, k)
        tot += len(set(a[o:o + t].tolist()) & set(b[o:o + t].tolist())) / t
    return tot / len(ks)


def calibrate_flat(run_plain, run_stop, ks, offsets, params, mean, inv_std, interval,
                   max_loss=0.005,
                   taus=(0.5, 0.6, 0.7, 0.8, 0.85, 0.9, 0.93, 0.95, 0.97, 0.98, 0.99, 0.995)):
    """calibrate() for a mixed stream: run_plain() and run_stop(model) return
    (flat ids, dists, stats); the smallest tau with agreement >= 1 - max_loss wins."""
    plain = run_plain()
    best = None
    table = []
    for tau in taus:
        got = run_stop(build_model(params, mean, inv_std, tau, interval))
        agree = agreement_flat(got[0], plain[0], ks, offsets)
        hops = float(got[2][:, 0].float().mean())
        table.append((tau, agree, hops))
        if best is None and agree >= 1.0 - max_loss:
            best = tau
    return (best if best is not None else 1.0), table
