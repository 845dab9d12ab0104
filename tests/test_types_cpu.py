"""uint32 and int64 keys and the stable argsort, on the CPU.

* the oracle's sorts of the new key types, pinned to numpy's sort (a
  library routine the oracle shares nothing with) on inputs where the
  plausible mistakes show: uint32 keys past 2^31 (a signed compare puts them
  first), int64 extremes (a missing or misplaced sign flip reorders them),
  many duplicates, sizes across the network bound;
* the oracle's argsort, pinned to numpy's stable argsort;
* the C ABI of the new entry points: declared, exported, argument errors
  before any device work, workspace sizes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    return hsort


@pytest.mark.parametrize("n", [0, 1, 2, 255, 256, 257, 5000, 100003])
def test_oracle_u32_against_numpy(oracle_mod, n):
    g = np.random.default_rng(n)
    a = g.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    if n > 4:
        a[:4] = [0, 2 ** 32 - 1, 2 ** 31, 2 ** 31 - 1]
    assert np.array_equal(oracle_mod.sort_u32(a), np.sort(a))
    d = g.integers(0, 8, n).astype(np.uint32) * np.uint32(0x40000001)  # few values, both halves of the range
    assert np.array_equal(oracle_mod.sort_u32(d), np.sort(d))


@pytest.mark.parametrize("n", [0, 1, 2, 255, 256, 257, 5000, 100003])
def test_oracle_i64_against_numpy(oracle_mod, n):
    g = np.random.default_rng(n + 1)
    a = g.integers(-2 ** 63, 2 ** 63 - 1, n, dtype=np.int64)
    if n > 6:
        a[:6] = [-2 ** 63, 2 ** 63 - 1, 0, -1, 1, -2 ** 32]
    assert np.array_equal(oracle_mod.sort_i64(a), np.sort(a))
    small = g.integers(-3, 3, n).astype(np.int64)  # values straddling zero, many duplicates
    assert np.array_equal(oracle_mod.sort_i64(small), np.sort(small))


@pytest.mark.parametrize("n", [0, 1, 7, 256, 257, 40000])
def test_oracle_argsort_against_numpy(oracle_mod, n):
    g = np.random.default_rng(n + 2)
    a = g.integers(-20, 20, n).astype(np.int32)  # heavy duplicates: stability matters
    k, idx = oracle_mod.argsort_i32(a)
    assert np.array_equal(idx, np.argsort(a, kind="stable").astype(np.int32))
    assert np.array_equal(k, np.sort(a))
    assert np.array_equal(a[idx], k)


def _declared():
    src = open(os.path.join(ROOT, "include", "hsort.h")).read()
    return re.findall(r"HS_API\s+[\w\s\*]*?\b(hs_\w+)\s*\(", src)


def test_new_entry_points_declared_and_exported(hs):
    names = set(_declared())
    for n in ("hs_sort_u32", "hs_sort_i64", "hs_argsort_i32"):
        assert n in names
        assert hasattr(hs.lib(), n)


def test_new_entry_points_argument_errors(hs):
    L = hs.lib()
    p = ctypes.c_void_p
    assert L.hs_sort_u32(None, 5, None, None, None) == -1
    assert L.hs_sort_u32(p(0x1000), -1, None, None, None) == -1
    assert L.hs_sort_i64(None, 3, None, None, None) == -1
    assert L.hs_sort_i64(p(0x1000), 1 << 31, None, None, None) == -1
    assert L.hs_sort_u32(p(0x1000), 1, None, None, None) == 0  # one key: nothing to do
    assert L.hs_sort_i64(None, 0, None, None, None) == 0
    assert L.hs_argsort_i32(None, p(0x1000), p(0x2000), 3, None, None, None) == -1
    assert L.hs_argsort_i32(p(0x1000), p(0x1000), None, 3, None, None, None) == -1
    # idx_out inside the keys, keys_out partly over keys
    assert L.hs_argsort_i32(p(0x1000), p(0x2000), p(0x2004), 3, None, None, None) == -1
    assert "overlap" in L.hs_last_error().decode()
    assert L.hs_argsort_i32(p(0x1000), p(0x1004), p(0x3000), 3, None, None, None) == -1
    assert L.hs_argsort_i32(None, None, None, 0, None, None, None) == 0


def test_new_ops_workspace(hs):
    n = 1 << 20
    assert hs.workspace_size(hs.OP_SORT_U32, n) == hs.workspace_size(hs.OP_SORT_I32, n)
    assert hs.workspace_size(hs.OP_SORT_I64, n) == hs.workspace_size(hs.OP_SORT_F64, n)


def test_binding_dtypes(hs):
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):  # CPU tensors are refused for every key type
        hs.sort_(torch.zeros(4, dtype=torch.uint32))
    with pytest.raises(ValueError):
        hs.sort_(torch.zeros(4, dtype=torch.int64))
    with pytest.raises(TypeError):
        hs.argsort(torch.zeros(4, dtype=torch.int64))
