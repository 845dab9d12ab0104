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


def ninther_adversary(m: int, span: int = 1024) -> np.ndarray:
    """int32 keys 0..m-1 arranged so that the on-chip sort's block levels
    peel only a few keys off a live range per level.

    McIlroy's adversary ("A Killer Adversary for Quicksort", 1999): keys are
    fixed lazily, the first time the pivot rule reads them; a key not yet
    fixed compares greater than every fixed one.  The pivot rule followed is
    the on-chip one for ranges longer than a span: the median of three
    medians of nine evenly spaced keys (positions b + (s-1)*i/8).  New keys
    are fixed in the order that puts the ninther at the fourth-smallest
    sample, so each level leaves a few keys below the pivot (a child of
    2..span keys, queued for a wave) and the rest above it: an 8192-key task
    takes about 900 block levels.  The block levels' three-
    way partition is stable (each class keeps the keys' order), which is what
    lets the construction follow the ranges from level to level.
    """
    val = [-1] * m
    nxt = 0
    arr = list(range(m))
    live = [(0, m)]
    rank_of_sample = [0, 1, 8, 2, 3, 7, 4, 5, 6]  # groups (0,1,8), (2,3,7), (4,5,6): medians 1, 3, 5
    while live:
        nl = []
        for b, e in live:
            s = e - b
            pos = [b + (s - 1) * i // 8 for i in range(9)]
            for _, el in sorted((rank_of_sample[k], arr[p]) for k, p in enumerate(pos) if val[arr[p]] < 0):
                if val[el] < 0:
                    val[el] = nxt
                    nxt += 1
            v = [val[arr[p]] for p in pos]
            med = [sorted(v[3 * g:3 * g + 3])[1] for g in range(3)]
            pv = sorted(med)[1]
            seg = arr[b:e]
            lt = [x for x in seg if 0 <= val[x] < pv]
            eq = [x for x in seg if val[x] == pv]
            gt = [x for x in seg if val[x] < 0 or val[x] > pv]
            arr[b:e] = lt + eq + gt
            rb = b + len(lt) + len(eq)
            if e - rb > span:
                nl.append((rb, e))
        live = nl
    for i in range(m):
        if val[i] < 0:
            val[i] = nxt
            nxt += 1
    return np.asarray(val, dtype=np.int32)
