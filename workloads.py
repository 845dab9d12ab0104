"""Seeded synthetic inputs shared by the tests, the smoke check and bench.py.

This module holds only random-number generation and array shaping; none of
the sort's arithmetic lives here, so the oracle and the HIP path can both be
fed from it without sharing any of the method's code.

The paper benchmarks "randomly generated values" (Sec. IV-A).  The recipes
below add the distributions of the workloads this library is measured on:
  * uniform int32 over the full range;
  * float64 uniform [0,1), standard normal, already sorted, reverse sorted;
  * int32 and float64 key/value pairs with 2^16 distinct keys (heavy
    duplicates) and the original index as value;
  * batched segments with log-uniform sizes;
  * float64 lognormal(0, 2), Zipf(1.1) ranks over 2^24 values, and an
    8-component Gaussian mixture.
All generators use numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_i32(n: int, seed: int = 1) -> np.ndarray:
    return rng(seed).integers(-(2 ** 31), 2 ** 31, size=n, dtype=np.int32)


def f64(n: int, dist: str = "uniform", seed: int = 2) -> np.ndarray:
    g = rng(seed)
    if dist == "uniform":
        return g.random(n)
    if dist == "normal":
        return g.standard_normal(n)
    if dist == "sorted":
        return np.sort(g.random(n))
    if dist == "reverse":
        return np.sort(g.random(n))[::-1].copy()
    if dist == "lognormal":
        return g.lognormal(0.0, 2.0, n)
    if dist == "zipf":
        return zipf_ranks(n, g).astype(np.float64)
    if dist == "mixture":
        return gauss_mixture(n, g)
    raise ValueError(dist)


def zipf_ranks(n: int, g: np.random.Generator, s: float = 1.1, nvals: int = 1 << 24) -> np.ndarray:
    """Ranks r in [1, nvals] with P(r) proportional to r^-s (inverse CDF)."""
    w = np.arange(1, nvals + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = g.random(n)
    return (np.searchsorted(cdf, u, side="right") + 1).clip(1, nvals)


def gauss_mixture(n: int, g: np.random.Generator, k: int = 8) -> np.ndarray:
    mu = g.uniform(-10.0, 10.0, k)
    sd = g.uniform(0.1, 2.0, k)
    c = g.integers(0, k, n)
    return mu[c] + sd[c] * g.standard_normal(n)


def kv_dup_i32(n: int, seed: int = 4, ndistinct: int = 1 << 16, force_extremes: bool = False):
    """Keys drawn from a table of `ndistinct` distinct int32; values = index."""
    g = rng(seed)
    if not 2 <= ndistinct <= (1 << 24):
        raise ValueError("ndistinct out of range")
    table = np.unique(g.integers(-(2 ** 31), 2 ** 31, size=2 * ndistinct + 64, dtype=np.int64))
    table = g.permutation(table)[:ndistinct]
    if table.size < ndistinct:
        raise ValueError("could not draw enough distinct keys")
    if force_extremes:
        table[0] = -(2 ** 31)
        table[-1] = 2 ** 31 - 1
    table = table.astype(np.int32)
    keys = table[g.integers(0, ndistinct, n)]
    vals = np.arange(n, dtype=np.int32)
    return keys, vals


def kv_dup_f64(n: int, seed: int = 6, ndistinct: int = 1 << 16, specials: bool = False):
    """float64 keys drawn from a table of `ndistinct` distinct N(0,1) values
    (with `specials`, the table's first entries are signed zeros, NaNs,
    infinities and denormals); values = index."""
    g = rng(seed)
    if not 2 <= ndistinct <= (1 << 24):
        raise ValueError("ndistinct out of range")
    table = np.unique(g.standard_normal(ndistinct + 64))
    table = g.permutation(table)[:ndistinct]
    if specials:
        s = f64_specials().view(np.uint64)  # NaN payloads copied as bits
        table.view(np.uint64)[:min(s.size, ndistinct)] = s[:ndistinct]
    keys = table[g.integers(0, ndistinct, n)]
    vals = np.arange(n, dtype=np.int32)
    return keys, vals


def segment_offsets(nseg: int, lo: int, hi: int, seed: int = 5) -> np.ndarray:
    """Offsets of nseg segments with sizes floor(exp(U(ln lo, ln hi)))."""
    g = rng(seed)
    sizes = np.floor(np.exp(g.uniform(np.log(lo), np.log(hi), nseg))).astype(np.int64)
    off = np.zeros(nseg + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def f64_specials() -> np.ndarray:
    """Signed zeros, infinities, NaNs of both signs, denormals, extremes."""
    bits = np.array([
        0x7FF8000000000000,  # +qNaN
        0xFFF8000000000000,  # -qNaN
        0x7FF0000000000001,  # +sNaN payload
        0xFFF0000000000001,  # -sNaN payload
        0x7FF0000000000000,  # +inf
        0xFFF0000000000000,  # -inf
        0x0000000000000000,  # +0
        0x8000000000000000,  # -0
        0x0000000000000001,  # +denorm_min
        0x8000000000000001,  # -denorm_min
        0x7FEFFFFFFFFFFFFF,  # +DBL_MAX
        0xFFEFFFFFFFFFFFFF,  # -DBL_MAX
        0x3FF0000000000000,  # 1.0
        0xBFF0000000000000,  # -1.0
    ], dtype=np.uint64)
    return bits.view(np.float64)
