"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no SquareSort arithmetic: it only draws keys.  Every
generator is a pure function of (n, seed) built on numpy's PCG64 stream, so
the GPU path and the CPU oracle always receive identical bytes.

Distributions:
  * the paper's four 32-bit experiment inputs (Section 4): a random
    permutation of 1..n, random binary values, uniform over 1..n, uniform
    over 1..sqrt(n);
  * random 64-bit values (the external-memory experiment, Section 4);
  * uniform u32 over [0, 2^32) or [0, 2^16) (heavy duplicates);
  * the key/value mixture: 80% Zipf(s=1.1) over 2^20 distinct random u64
    values, 10% one constant random u64, 10% an ascending run of random u64
    with 1% of its positions swapped with random partners inside the run;
    value = original index.
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_u32(n: int, seed: int, hi: int = 1 << 32) -> np.ndarray:
    """i.i.d. uniform over [0, hi)."""
    return _rng(seed).integers(0, hi, size=n, dtype=np.uint64).astype(np.uint32)


def uniform_u64(n: int, seed: int) -> np.ndarray:
    return _rng(seed).integers(0, 1 << 64, size=n, dtype=np.uint64)


def paper_u32(kind: str, n: int, seed: int) -> np.ndarray:
    """The four input families of the paper's experiments (values >= 1)."""
    g = _rng(seed)
    if kind == "perm":
        return (g.permutation(n) + 1).astype(np.uint32)
    if kind == "binary":
        return g.integers(0, 2, size=n, dtype=np.uint32)
    if kind == "uniform_n":
        return g.integers(1, max(n, 1) + 1, size=n, dtype=np.uint64).astype(np.uint32)
    if kind == "uniform_sqrt":
        r = max(1, math.isqrt(max(n, 1)))
        return g.integers(1, r + 1, size=n, dtype=np.uint64).astype(np.uint32)
    raise ValueError(kind)


def zipf_table(num_values: int, s: float) -> np.ndarray:
    """Cumulative distribution of ranks 1..num_values with P(r) ~ r^-s."""
    w = np.arange(1, num_values + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def kv_mixture(n: int, seed: int, zipf_values: int = 1 << 20, s: float = 1.1):
    """Key/value mixture; returns (keys u64, values u32 = original index)."""
    g = _rng(seed)
    n_zipf = (8 * n) // 10
    n_const = n // 10
    n_run = n - n_zipf - n_const
    distinct = g.integers(0, 1 << 64, size=zipf_values, dtype=np.uint64)
    cdf = zipf_table(zipf_values, s)
    ranks = np.searchsorted(cdf, g.random(n_zipf), side="right")
    ranks = np.minimum(ranks, zipf_values - 1)
    keys = np.empty(n, np.uint64)
    keys[:n_zipf] = distinct[ranks]
    keys[n_zipf:n_zipf + n_const] = g.integers(0, 1 << 64, dtype=np.uint64)
    run = np.sort(g.integers(0, 1 << 64, size=n_run, dtype=np.uint64))
    n_swap = n_run // 100
    if n_swap:
        a = g.choice(n_run, size=n_swap, replace=False)
        b = g.integers(0, n_run, size=n_swap)
        for i, j in zip(a.tolist(), b.tolist()):
            run[i], run[j] = run[j], run[i]
    keys[n_zipf + n_const:] = run
    vals = np.arange(n, dtype=np.uint32)
    return keys, vals


def log_uniform_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Instance sizes log-uniform in [lo, hi] (batched and served forms)."""
    g = _rng(seed)
    e = g.uniform(math.log(lo), math.log(hi), size=count)
    return np.clip(np.exp(e).astype(np.int64), lo, hi)


def zipf_keys(n: int, seed: int, bits: int = 32, num_values: int = 1 << 20, s: float = 1.1) -> np.ndarray:
    """n keys drawn Zipf(s) over num_values distinct random values of `bits`
    bits (rank r with probability proportional to r^-s)."""
    g = _rng(seed)
    distinct = g.integers(0, 1 << bits, size=num_values, dtype=np.uint64)
    ranks = np.minimum(np.searchsorted(zipf_table(num_values, s), g.random(n), side="right"), num_values - 1)
    keys = distinct[ranks]
    return keys.astype(np.uint32) if bits == 32 else keys


def serve_requests(count: int, seed: int, lo: int = 1 << 12, hi: int = 1 << 24):
    """Request mix of the served form: sizes log-uniform in [lo, hi]; 70%
    uint32 keys, 30% (uint64 key, uint32 value = index) pairs; keys uniform or
    Zipf(1.1) over 2^20 values with probability 1/2 each.  Returns a list of
    dicts (kind, n, dist, data_seed, seed) and the keys/values of each."""
    g = _rng(seed)
    sizes = log_uniform_sizes(count, lo, hi, seed + 1)
    kinds = np.where(g.random(count) < 0.7, "u32", "kv")
    dists = np.where(g.random(count) < 0.5, "uniform", "zipf")
    reqs = []
    for i in range(count):
        n, kind, dist = int(sizes[i]), str(kinds[i]), str(dists[i])
        ds = seed * 100_003 + i
        if kind == "u32":
            keys = uniform_u32(n, ds) if dist == "uniform" else zipf_keys(n, ds, 32)
            vals = None
        else:
            keys = uniform_u64(n, ds) if dist == "uniform" else zipf_keys(n, ds, 64)
            vals = np.arange(n, dtype=np.uint32)
        reqs.append({"id": i, "kind": kind, "n": n, "dist": dist, "data_seed": ds, "seed": i + 1,
                     "keys": keys, "vals": vals})
    return reqs
