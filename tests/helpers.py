"""Checkers shared by the tests (no sort arithmetic: only verification)."""
from __future__ import annotations

import numpy as np


def insertion_sort(xs):
    """Textbook insertion sort, used as brute force on tiny inputs."""
    a = list(xs)
    for i in range(1, len(a)):
        x = a[i]
        j = i - 1
        while j >= 0 and a[j] > x:
            a[j + 1] = a[j]
            j -= 1
        a[j + 1] = x
    return a


def is_sorted(a: np.ndarray) -> bool:
    return a.size < 2 or bool(np.all(a[:-1] <= a[1:]))


def kv_index_check(keys_in: np.ndarray, keys_out: np.ndarray, vals_out: np.ndarray) -> None:
    """Exact pair check when the input values are the original indices:
    vals_out must be a permutation of 0..n-1 and keys_in[vals_out] == keys_out."""
    n = keys_in.size
    assert vals_out.size == n and keys_out.size == n
    idx = vals_out.astype(np.int64)
    assert np.all((idx >= 0) & (idx < n)), "value out of range"
    seen = np.zeros(n, dtype=bool)
    seen[idx] = True
    assert seen.all(), "values are not a permutation"
    assert np.array_equal(keys_in[idx], keys_out), "a key lost its value"


def pair_multiset_equal(k0, v0, k1, v1) -> bool:
    a = np.sort((k0.astype(np.int64) << 32) | (v0.astype(np.int64) & 0xFFFFFFFF))
    b = np.sort((k1.astype(np.int64) << 32) | (v1.astype(np.int64) & 0xFFFFFFFF))
    return bool(np.array_equal(a, b))
