"""hs_sort_i32_noalloc (static device scratch, no allocation) against the
existing entry point hs_sort_i32 and the oracle, through the C ABI: several
calls in a row on one GPU, each smaller than the one before it (the later
calls find the earlier calls' contents in the shared scratch), then sizes
that take the one-workgroup and one-wave paths, and the size limit."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MAX_N = 1 << 22


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hsort


def test_noalloc_matches_hs_sort_i32(hs, oracle_mod):
    L = hs.lib()
    stream = torch.cuda.current_stream().cuda_stream
    for r, n in enumerate([MAX_N, 3000017, 100003, 5000, 777, 2]):
        print(f"noalloc call {r}: n={n}", flush=True)
        a = workloads.uniform_i32(n, seed=200 + r)
        x = torch.from_numpy(a).to("cuda")
        y = x.clone()
        assert L.hs_sort_i32_noalloc(ctypes.c_void_p(x.data_ptr()), n, ctypes.c_void_p(stream)) == 0, \
            L.hs_last_error()
        assert L.hs_sort_i32(ctypes.c_void_p(y.data_ptr()), n, None, None, ctypes.c_void_p(stream)) == 0
        got = x.cpu().numpy()
        assert np.array_equal(got, y.cpu().numpy()), f"call {r}: differs from hs_sort_i32"
        assert np.array_equal(got, oracle_mod.sort_i32(a)), f"call {r}: differs from the oracle"


def test_noalloc_duplicates_and_limits(hs, oracle_mod):
    L = hs.lib()
    stream = torch.cuda.current_stream().cuda_stream
    k, _ = workloads.kv_dup_i32(1 << 21, seed=210, ndistinct=7)
    x = torch.from_numpy(k).to("cuda")
    assert L.hs_sort_i32_noalloc(ctypes.c_void_p(x.data_ptr()), k.size, ctypes.c_void_p(stream)) == 0
    assert np.array_equal(x.cpu().numpy(), oracle_mod.sort_i32(k))
    big = torch.empty(MAX_N + 1, dtype=torch.int32, device="cuda")
    assert L.hs_sort_i32_noalloc(ctypes.c_void_p(big.data_ptr()), MAX_N + 1, ctypes.c_void_p(stream)) == -1
    assert "static scratch" in L.hs_last_error().decode()
    assert L.hs_sort_i32_noalloc(None, 0, ctypes.c_void_p(stream)) == 0
