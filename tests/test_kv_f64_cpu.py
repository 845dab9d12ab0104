"""Key/value pairs with float64 keys, on the CPU.

* the oracle's pair sort, pinned to numpy (a library routine the oracle
  shares nothing with): the keys come out as numpy's sort of the same
  numbers, bit for bit, and the (key bits, value) pairs are the input's
  multiset -- on inputs where the plausible mistakes show (values left
  behind by a swap, NaNs, signed zeros, infinities and denormals under
  totalOrder, heavy duplicates, sizes across the network bound);
* brute force on tiny inputs: a textbook insertion sort of the pairs by the
  totalOrder key of the IEEE special-value table;
* the C ABI of hs_sort_kv_f64: declared, exported, argument errors before
  any device work (the overlap check spans 8-byte keys), workspace sizes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads
from helpers import insertion_sort

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    return hsort


def _pairs(bits, vals):
    """The pairs as a sorted structured array (key bits, value bits)."""
    a = np.empty(bits.size, dtype=[("k", np.uint64), ("v", np.uint32)])
    a["k"] = bits
    a["v"] = vals.view(np.uint32)
    return np.sort(a, order=["k", "v"])


@pytest.mark.parametrize("n", [0, 1, 2, 255, 256, 257, 5000, 100003])
def test_oracle_kv_f64_against_numpy(oracle_mod, n):
    """No NaNs or zeros: totalOrder is the numeric order and numpy's sort
    fixes the key sequence; the pairs must be the input's."""
    keys, vals = workloads.kv_dup_f64(n, seed=n + 3, ndistinct=max(2, min(n // 8, 1 << 16)))
    ko, vo = oracle_mod.sort_kv_f64(keys, vals)
    assert np.array_equal(ko.view(np.uint64), np.sort(keys).view(np.uint64))
    assert np.array_equal(_pairs(ko.view(np.uint64), vo), _pairs(keys.view(np.uint64), vals))
    # with the values being the input positions, each one still sits beside its key
    assert np.array_equal(keys[vo].view(np.uint64), ko.view(np.uint64))


def test_oracle_kv_f64_specials(oracle_mod):
    """NaNs of both signs, infinities, signed zeros and denormals as keys:
    the key sequence is the golden totalOrder table, each entry repeated,
    and every value stays with its key."""
    table = [int(r.split()[0], 16) for r in open(os.path.join(ROOT, "tests", "golden",
                                                             "ieee754_total_order.txt"))
             if r.strip() and not r.startswith("#")]
    expect = np.repeat(np.array(table, dtype=np.uint64), 7)
    g = workloads.rng(11)
    perm = g.permutation(expect.size)
    bits = expect[perm]
    vals = np.arange(bits.size, dtype=np.int32)
    ko, vo = oracle_mod.sort_kv_f64(bits.view(np.float64), vals)
    assert np.array_equal(ko.view(np.uint64), expect)
    assert np.array_equal(bits[vo], ko.view(np.uint64))


@pytest.mark.parametrize("seed", range(6))
def test_oracle_kv_f64_brute_force(oracle_mod, seed):
    """Tiny inputs from the special-value table: insertion sort of (totalOrder
    rank, value) pairs decides the keys; the pairs must match as a multiset."""
    table = [int(r.split()[0], 16) for r in open(os.path.join(ROOT, "tests", "golden",
                                                             "ieee754_total_order.txt"))
             if r.strip() and not r.startswith("#")]
    rank = {b: i for i, b in enumerate(table)}
    g = workloads.rng(100 + seed)
    for n in (0, 1, 2, 3, 5, 8, 13, 31):
        pick = g.integers(0, len(table), n)
        bits = np.array([table[i] for i in pick], dtype=np.uint64)
        vals = g.integers(-5, 5, n).astype(np.int32)
        want = insertion_sort([(rank[int(b)], int(b)) for b in bits])
        for leaf in (1, 4, 256):
            ko, vo = oracle_mod.sort_kv_f64(bits.view(np.float64), vals, leaf=leaf)
            assert [int(b) for b in ko.view(np.uint64)] == [b for _, b in want]
            assert np.array_equal(_pairs(ko.view(np.uint64), vo), _pairs(bits, vals))


def test_kv_f64_declared_and_exported(hs):
    src = open(os.path.join(ROOT, "include", "hsort.h")).read()
    assert "hs_sort_kv_f64" in re.findall(r"HS_API\s+[\w\s\*]*?\b(hs_\w+)\s*\(", src)
    assert hasattr(hs.lib(), "hs_sort_kv_f64")


def test_kv_f64_argument_errors(hs):
    L = hs.lib()
    p = ctypes.c_void_p
    assert L.hs_sort_kv_f64(None, p(0x8000), 3, None, None, None) == -1
    assert L.hs_sort_kv_f64(p(0x1000), None, 3, None, None, None) == -1
    assert L.hs_sort_kv_f64(p(0x1000), p(0x8000), -1, None, None, None) == -1
    assert L.hs_sort_kv_f64(p(0x1000), p(0x8000), 1 << 31, None, None, None) == -1
    # three 8-byte keys end at 0x1018: values at 0x1010 overlap them (a 4-byte
    # stride would have missed it)
    assert L.hs_sort_kv_f64(p(0x1000), p(0x1010), 3, None, None, None) == -1
    assert "overlap" in L.hs_last_error().decode()
    assert L.hs_sort_kv_f64(p(0x1000), p(0x8000), 1, None, None, None) == 0  # one pair
    assert L.hs_sort_kv_f64(None, None, 0, None, None, None) == 0


def test_kv_f64_workspace(hs):
    n = 1 << 20
    ws = hs.workspace_size(hs.OP_SORT_KV_F64, n)
    assert ws >= 2 * 16 * n  # two 16-byte words per pair: the ping-pong buffers
    assert ws > hs.workspace_size(hs.OP_SORT_KV_I32, n)
    # the learned front end adds its sample (8-byte keys and their values), model and histograms
    assert hs.workspace_size(hs.OP_SORT_KV_F64, n, opts=hs.learned_opts()) > ws + 12 * (1 << 16)


def test_kv_f64_binding_dtypes(hs):
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):  # CPU tensors are refused
        hs.sort_kv_(torch.zeros(4, dtype=torch.float64), torch.zeros(4, dtype=torch.int32))
    with pytest.raises(TypeError):
        hs.sort_kv_(torch.zeros(4, dtype=torch.float32), torch.zeros(4, dtype=torch.int32))


def test_kv_dup_f64_recipe():
    """The float64 key/value inputs: the requested number of distinct keys,
    values = positions, and the special keys kept bit for bit (NaN payloads
    and signed zeros included)."""
    keys, vals = workloads.kv_dup_f64(200000, seed=9, ndistinct=1000)
    assert np.unique(keys.view(np.uint64)).size == 1000
    assert np.array_equal(vals, np.arange(200000, dtype=np.int32))
    keys, _ = workloads.kv_dup_f64(50000, seed=9, ndistinct=40, specials=True)
    specials = set(int(b) for b in workloads.f64_specials().view(np.uint64))
    assert specials <= set(int(b) for b in np.unique(keys.view(np.uint64)))


@pytest.mark.parametrize("n", [0, 1, 2, 257, 40000])
def test_oracle_argsort_f64_against_numpy(oracle_mod, n):
    """Without NaNs and zeros totalOrder is the numeric order, so numpy's
    stable argsort decides every position (heavy duplicates: stability
    matters)."""
    keys, _ = workloads.kv_dup_f64(n, seed=n + 5, ndistinct=max(2, n // 50))
    k, idx = oracle_mod.argsort_f64(keys)
    want = np.argsort(keys, kind="stable").astype(np.int32)
    assert np.array_equal(idx, want)
    assert np.array_equal(k.view(np.uint64), keys[want].view(np.uint64))


def test_oracle_argsort_f64_brute_force(oracle_mod):
    """Special keys: insertion sort of (totalOrder rank, position) pairs."""
    table = [int(r.split()[0], 16) for r in open(os.path.join(ROOT, "tests", "golden",
                                                             "ieee754_total_order.txt"))
             if r.strip() and not r.startswith("#")]
    rank = {b: i for i, b in enumerate(table)}
    g = workloads.rng(7)
    for n in (1, 2, 5, 9, 30):
        bits = np.array([table[i] for i in g.integers(0, len(table), n)], dtype=np.uint64)
        want = [p for _, p in insertion_sort([(rank[int(b)], p) for p, b in enumerate(bits)])]
        for leaf in (1, 256):
            _, idx = oracle_mod.argsort_f64(bits.view(np.float64), leaf=leaf)
            assert list(idx) == want


def test_argsort_f64_abi(hs):
    L = hs.lib()
    p = ctypes.c_void_p
    assert hasattr(L, "hs_argsort_f64")
    assert L.hs_argsort_f64(None, p(0x1000), p(0x8000), 3, None, None, None) == -1
    # idx_out inside keys_out (8-byte keys: 3 of them end at 0x1018)
    assert L.hs_argsort_f64(p(0x4000), p(0x1000), p(0x1010), 3, None, None, None) == -1
    assert "overlap" in L.hs_last_error().decode()
    assert L.hs_argsort_f64(None, None, None, 0, None, None, None) == 0
