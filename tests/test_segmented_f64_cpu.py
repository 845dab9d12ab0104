"""Batched (segmented) sorts of float64 keys, on the CPU: the oracle pinned
to numpy's sort of each segment, and the C ABI of hs_sort_segmented_f64."""
import ctypes

import numpy as np
import pytest

import workloads


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    return hsort


@pytest.mark.parametrize("nseg", [1, 7, 300])
def test_oracle_segmented_f64_against_numpy(oracle_mod, nseg):
    off = workloads.segment_offsets(nseg, 1, 5000, seed=nseg).astype(np.int64)
    keys = workloads.f64(int(off[-1]), "normal", seed=nseg)
    got = oracle_mod.sort_segmented_f64(keys, off)
    for i in range(nseg):
        a, b = off[i], off[i + 1]
        assert np.array_equal(got[a:b].view(np.uint64), np.sort(keys[a:b]).view(np.uint64))


def test_segmented_f64_abi(hs):
    L = hs.lib()
    p = ctypes.c_void_p
    assert hasattr(L, "hs_sort_segmented_f64")
    assert L.hs_sort_segmented_f64(p(0x1000), 10, None, 2, None, None, None) == -1  # offsets missing
    assert L.hs_sort_segmented_f64(None, 10, p(0x2000), 2, None, None, None) == -1  # keys missing
    assert L.hs_sort_segmented_f64(p(0x1000), 10, p(0x2000), -1, None, None, None) == -1
    assert L.hs_sort_segmented_f64(p(0x1000), 10, p(0x2000), 0, None, None, None) == 0  # no segments
    n = 1 << 20
    assert hs.workspace_size(hs.OP_SORT_SEGMENTED_F64, n, 1000) >= hs.workspace_size(hs.OP_SORT_F64, n)
