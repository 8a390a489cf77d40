"""Seeded synthetic workloads shaped like the paper's datasets (Sec. 6.1, Table "datasets").

This module only draws random numbers. It holds none of the search method's
arithmetic, so both the CPU oracle's tests and the GPU path use it to get the
same inputs. Every array is float32 (vectors) or int32/int64 (ids).

Each workload has three independent numpy PCG64 streams:
  base seed  = 10*cfg + 1   (cluster centres, base vectors)
  query seed = 10*cfg + 2   (held-out queries, query descriptors)
  train seed = 10*cfg + 3   (extra queries used to train the learned stop)

Workloads (the paper's datasets are not available; these stand in for them):
  cfg1  10,000 x 128, integer-valued Gaussian mixture (64 clusters), L2
  cfg2  1,000,000 x 128, same generator with 1,000 clusters (SIFT1M-shaped), L2
  cfg3  1,183,514 x 100, unit vectors, Zipf(1.1) cluster sizes (GloVe-shaped), IP
  cfg4  95,000 x 1,369, 80% zeros, lognormal non-zeros (Enron-shaped), L2
  cfg5  2,000,000 x 300, anisotropic mixture (2,000 clusters), L2, mixed stream
"""
from __future__ import annotations

import numpy as np

_CHUNK = 65536  # rows drawn per call; fixed so the stream order never changes


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# integer-valued isotropic mixture (cfg1, cfg2)
# --------------------------------------------------------------------------
def _int_mixture_centres(rng, n_clusters, dim):
    return rng.uniform(0.0, 100.0, size=(n_clusters, dim))


def _int_mixture_draw(rng, centres, n, sigma=10.0):
    dim = centres.shape[1]
    z = rng.integers(0, centres.shape[0], size=n)
    out = np.empty((n, dim), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        x = centres[z[s:e]] + sigma * rng.standard_normal(size=(e - s, dim))
        out[s:e] = np.clip(np.rint(x), 0.0, 255.0).astype(np.float32)
    return out


def int_mixture(cfg: int, n_base: int, n_query: int, n_clusters: int, dim: int = 128,
                n_train: int = 0):
    """Base, query (and optional training-query) sets of the integer mixture.

    Centres ~ U[0,100]^dim, uniform cluster choice, x = clip(rint(c + 10 N(0,I)), 0, 255).
    """
    rb = _rng(10 * cfg + 1)
    centres = _int_mixture_centres(rb, n_clusters, dim)
    base = _int_mixture_draw(rb, centres, n_base)
    queries = _int_mixture_draw(_rng(10 * cfg + 2), centres, n_query)
    if n_train:
        train = _int_mixture_draw(_rng(10 * cfg + 3), centres, n_train)
        return base, queries, train
    return base, queries


def cfg1(n_base=10_000, n_query=1_000, n_train=0):
    return int_mixture(1, n_base, n_query, 64, 128, n_train)


def cfg2(n_base=1_000_000, n_query=10_000, n_train=0):
    return int_mixture(2, n_base, n_query, 1000, 128, n_train)


# --------------------------------------------------------------------------
# unit-norm Zipf mixture (cfg3, inner product, indexed queries)
# --------------------------------------------------------------------------
def cfg3(n_base=1_183_514, n_query=10_000, dim=100, n_clusters=1000, sigma=0.1):
    """Unit vectors around 1,000 unit centres with Zipf(1.1) cluster weights.

    Queries are n_query distinct base ids (each is searched from itself).
    """
    rb = _rng(31)
    mu = rb.standard_normal(size=(n_clusters, dim))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    w = np.arange(1, n_clusters + 1, dtype=np.float64) ** -1.1
    w /= w.sum()
    z = rb.choice(n_clusters, size=n_base, p=w)
    base = np.empty((n_base, dim), dtype=np.float32)
    for s in range(0, n_base, _CHUNK):
        e = min(n_base, s + _CHUNK)
        x = mu[z[s:e]] + sigma * rb.standard_normal(size=(e - s, dim))
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        base[s:e] = x.astype(np.float32)
    qids = _rng(32).choice(n_base, size=n_query, replace=False).astype(np.int32)
    return base, qids


# --------------------------------------------------------------------------
# sparse lognormal (cfg4)
# --------------------------------------------------------------------------
def _sparse_lognormal(rng, n, dim, p_zero=0.8):
    out = np.empty((n, dim), dtype=np.float32)
    for s in range(0, n, _CHUNK // 8):
        e = min(n, s + _CHUNK // 8)
        nz = rng.random(size=(e - s, dim)) >= p_zero
        v = np.exp(rng.standard_normal(size=(e - s, dim)))
        out[s:e] = np.where(nz, v, 0.0).astype(np.float32)
    return out


def cfg4(n_base=95_000, n_query=5_000, dim=1369):
    base = _sparse_lognormal(_rng(41), n_base, dim)
    queries = _sparse_lognormal(_rng(42), n_query, dim)
    return base, queries


# --------------------------------------------------------------------------
# anisotropic mixture + mixed query stream (cfg5)
# --------------------------------------------------------------------------
def _aniso_draw(rng, centres, sig, n):
    dim = centres.shape[1]
    z = rng.integers(0, centres.shape[0], size=n)
    out = np.empty((n, dim), dtype=np.float32)
    for s in range(0, n, _CHUNK // 2):
        e = min(n, s + _CHUNK // 2)
        zz = z[s:e]
        out[s:e] = (centres[zz] + sig[zz] * rng.standard_normal(size=(e - s, dim))).astype(np.float32)
    return out


def cfg5(n_base=2_000_000, n_query=100_000, dim=300, n_clusters=2000, n_train=0):
    """Base set plus a mixed descriptor stream.

    Returns base, queries (n_query x dim, fresh vectors), and a dict of
    per-descriptor fields: k in {1,10,100}, eps in {0,0.1,0.2}, indexed flag
    (Bernoulli 0.5) and, for indexed descriptors, a random base id.
    """
    rb = _rng(51)
    centres = rb.uniform(0.0, 100.0, size=(n_clusters, dim))
    sig = rb.uniform(0.5, 2.0, size=(n_clusters, dim))
    base = _aniso_draw(rb, centres, sig, n_base)
    rq = _rng(52)
    queries = _aniso_draw(rq, centres, sig, n_query)
    desc = {
        "k": rq.choice(np.array([1, 10, 100], dtype=np.int32), size=n_query),
        "eps": rq.choice(np.array([0.0, 0.1, 0.2], dtype=np.float32), size=n_query),
        "indexed": (rq.random(size=n_query) < 0.5).astype(np.int32),
        "vertex": rq.integers(0, n_base, size=n_query).astype(np.int32),
    }
    if n_train:
        train = _aniso_draw(_rng(53), centres, sig, n_train)
        return base, queries, desc, train
    return base, queries, desc


# --------------------------------------------------------------------------
# small random inputs for unit tests
# --------------------------------------------------------------------------
def small_int(seed: int, n: int, dim: int, hi: int = 16):
    """Tiny integer-valued sets (lots of exact distance ties)."""
    return _rng(1000 + seed).integers(0, hi, size=(n, dim)).astype(np.float32)


def small_float(seed: int, n: int, dim: int):
    return _rng(2000 + seed).standard_normal(size=(n, dim)).astype(np.float32)


def small_unit(seed: int, n: int, dim: int):
    x = _rng(3000 + seed).standard_normal(size=(n, dim))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x.astype(np.float32)


def rng(seed: int) -> np.random.Generator:
    """A generator for tests that need extra random draws (ids, permutations)."""
    return _rng(5000 + seed)
