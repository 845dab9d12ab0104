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


def median3_adversary(m: int, span: int = 1024) -> np.ndarray:
    """int32 keys 0..m-1 arranged so that the on-chip sort's block levels,
    run with the paper's 3-value pivot (HS_PIVOT_MEDIAN3: the median of the
    first, middle and last key of a range, Sec. IV-A), peel only a few keys
    off the live range per level.

    McIlroy's adversary ("A Killer Adversary for Quicksort", 1999): keys are
    fixed lazily, the first time the pivot rule reads them; a key not yet
    fixed compares greater than every fixed one.  Each level fixes the
    range's unfixed samples to the next smallest values, so the median is
    one of the smallest keys of the range: the keys below it (a child of
    2..span keys, queued for a wave) leave, the rest stays live.  The block
    levels' split keeps the keys' order within each class (two classes, < p
    and >= p, when some key is below the pivot and fewer than 1/32 of the
    range equal it, else three: < p, == p, > p), which is what lets the
    construction follow the ranges from level to level: an 8192-key task
    takes thousands of block levels.
    """
    val = [-1] * m
    nxt = 0
    arr = list(range(m))
    live = [(0, m)]
    while live:
        nl = []
        for b, e in live:
            s = e - b
            for p in (b, e - 1, b + (s - 1) // 2):
                if val[arr[p]] < 0:
                    val[arr[p]] = nxt
                    nxt += 1
            pv = sorted(val[arr[p]] for p in (b, b + (s - 1) // 2, e - 1))[1]
            seg = arr[b:e]
            lt = [x for x in seg if 0 <= val[x] < pv]
            eq = [x for x in seg if val[x] == pv]
            gt = [x for x in seg if val[x] < 0 or val[x] > pv]
            if len(lt) == 0 or 32 * len(eq) >= s:
                arr[b:e] = lt + eq + gt
                rb = b + len(lt) + len(eq)
            else:
                arr[b:e] = lt + [x for x in seg if not (0 <= val[x] < pv)]
                rb = b + len(lt)
            if len(lt) > span:
                nl.append((b, b + len(lt)))
            if e - rb > span:
                nl.append((rb, e))
        live = nl
    for i in range(m):
        if val[i] < 0:
            val[i] = nxt
            nxt += 1
    return np.asarray(val, dtype=np.int32)
