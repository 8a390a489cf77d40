"""Host-side evaluation of search results (Sec. 2.1, Eq. recall@k)."""
from __future__ import annotations

import numpy as np


def recall_at_k(ids, gt_ids, k: int) -> float:
    """Mean over queries of |ANNS(q) n KNN(q)| / k, using the first k of each."""
    ids = np.asarray(ids)[:, :k]
    gt = np.asarray(gt_ids)[:, :k]
    hits = 0
    for a, b in zip(ids, gt):
        hits += len(set(a[a >= 0].tolist()) & set(b.tolist()))
    return hits / (k * ids.shape[0]) if ids.shape[0] else 0.0


def recall_tie_aware(ids, dists_true_of_ids, gt_dists, k: int) -> float:
    """A returned vertex counts when its true distance is within the true k-th
    distance (exact ties at rank k are common on integer data)."""
    ids = np.asarray(ids)[:, :k]
    d = np.asarray(dists_true_of_ids)[:, :k]
    kth = np.asarray(gt_dists)[:, k - 1:k]
    ok = (ids >= 0) & (d <= kth)
    return float(ok.sum()) / (k * ids.shape[0]) if ids.shape[0] else 0.0
