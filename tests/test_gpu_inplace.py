"""Partition levels in place (hs_opts.inplace = 1) on the GPU, against the oracle.

The sorted output is unique, so every format must come out bit-identical to
the oracle's (key/value: identical keys, the pairs' multiset, and the
library's tie rule), whichever way the levels moved the keys.  Sizes span
many tiles with ragged tails; a low on-chip limit forces deep recursion with
many small segments per level (partial tiles at both ends of most of them);
few distinct keys exercise the equal-key rule (strict segments and fills).
The partition entry point is checked against Algorithm 3's contract.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hsort


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _ip(hs, local_T=0):
    o = hs.Opts()
    o.inplace = 1
    o.local_T = local_T
    return o


@pytest.mark.parametrize("n", [8193, 100003, (1 << 20) + 7, (1 << 22) + 3])
@pytest.mark.parametrize("local_T", [0, 700])
def test_inplace_i32_f64(hs, oracle_mod, n, local_T):
    print(f"inplace i32/f64 n={n} T={local_T}", flush=True)
    a = workloads.uniform_i32(n, seed=n)
    t = _gpu(a)
    hs.sort_(t, opts=_ip(hs, local_T))
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i32(a))
    f = workloads.f64(n, "normal", seed=n + 1)
    t = _gpu(f)
    hs.sort_(t, opts=_ip(hs, local_T))
    assert np.array_equal(t.cpu().numpy().view(np.uint64), oracle_mod.sort_f64(f).view(np.uint64))


# The classify pass gives each workgroup (one per compute unit) a contiguous
# run of ceil(tiles / workgroups) tiles of a level and has the loads of the
# two tiles after the current one in flight, past the run's end too.  A
# first level of one tile more than a multiple of the workgroup count leaves
# runs of two or three tiles, one workgroup with a single tile and others
# with none.
@pytest.mark.parametrize("mult", [1, 2])
def test_inplace_tile_runs(hs, oracle_mod, mult):
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    n = mult * ncu * 16384 + 1  # int32: 16384-key tiles
    print(f"inplace tile runs i32 n={n}", flush=True)
    a = workloads.uniform_i32(n, seed=40 + mult)
    t = _gpu(a)
    hs.sort_(t, opts=_ip(hs))
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i32(a))
    n = mult * ncu * 8192 + 1  # float64: 8192-key tiles
    print(f"inplace tile runs f64 n={n}", flush=True)
    f = workloads.f64(n, "uniform", seed=50 + mult)
    t = _gpu(f)
    hs.sort_(t, opts=_ip(hs))
    assert np.array_equal(t.cpu().numpy().view(np.uint64), oracle_mod.sort_f64(f).view(np.uint64))


def test_inplace_duplicates_and_specials(hs, oracle_mod):
    g = workloads.rng(3)
    for n, nd in ((300007, 5), (200003, 1)):
        a = g.integers(-nd, nd + 1, n).astype(np.int32)
        t = _gpu(a)
        hs.sort_(t, opts=_ip(hs, 1000))
        assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i32(a))
    keys, _ = workloads.kv_dup_f64(250001, seed=5, ndistinct=40, specials=True)
    t = _gpu(keys)
    hs.sort_(t, opts=_ip(hs))
    assert np.array_equal(t.cpu().numpy().view(np.uint64), oracle_mod.sort_f64(keys).view(np.uint64))


@pytest.mark.parametrize("kind", ["kv_i32", "kv_f64", "u32", "i64"])
def test_inplace_other_formats(hs, oracle_mod, kind):
    n = 400009
    if kind == "kv_i32":
        k, v = workloads.kv_dup_i32(n, seed=6, ndistinct=5000)
        tk, tv = _gpu(k), _gpu(v)
        hs.sort_kv_(tk, tv, opts=_ip(hs, 2000))
        ok, _ = oracle_mod.sort_kv_i32(k, v)
        ko, vo = tk.cpu().numpy(), tv.cpu().numpy()
        assert np.array_equal(ko, ok) and np.array_equal(k[vo], ko)
    elif kind == "kv_f64":
        k, _ = workloads.kv_dup_f64(n, seed=7, ndistinct=3000, specials=True)
        v = workloads.rng(8).integers(-(2 ** 31), 2 ** 31, n, dtype=np.int64).astype(np.int32)
        tk, tv = _gpu(k), _gpu(v)
        hs.sort_kv_(tk, tv, opts=_ip(hs))
        order = np.lexsort((v.view(np.uint32), oracle_mod.f64_order_keys(k)))
        ok, _ = oracle_mod.sort_kv_f64(k, v)
        assert np.array_equal(tk.cpu().numpy().view(np.uint64), ok.view(np.uint64))
        assert np.array_equal(tv.cpu().numpy(), v[order])
    elif kind == "u32":
        a = workloads.rng(9).integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
        t = _gpu(a)
        hs.sort_(t, opts=_ip(hs))
        assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_u32(a))
    else:
        a = workloads.rng(10).integers(-2 ** 63, 2 ** 63 - 1, n, dtype=np.int64)
        t = _gpu(a)
        hs.sort_(t, opts=_ip(hs, 1500))
        assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i64(a))


def test_inplace_segmented(hs, oracle_mod):
    off = workloads.segment_offsets(3000, 16, 1 << 16, seed=11).astype(np.int64)
    keys = workloads.uniform_i32(int(off[-1]), seed=12)
    t = _gpu(keys)
    hs.sort_segmented_(t, _gpu(off), opts=_ip(hs, 1000))
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_segmented_i32(keys, off))


@pytest.mark.parametrize("n", [1, 64, 16385, (1 << 20) + 9])
def test_inplace_partition(hs, oracle_mod, n):
    a = workloads.uniform_i32(n, seed=n + 20)
    for pivot in (0, int(a[n // 2]), -(2 ** 31), 2 ** 31 - 1):
        t = _gpu(a)
        cnt = int(hs.partition_(t, pivot, opts=_ip(hs)).cpu().item())
        got = t.cpu().numpy()
        _, want = oracle_mod.partition_le_i32(a, pivot)
        assert cnt == want
        assert np.all(got[:cnt] <= pivot) and np.all(got[cnt:] > pivot)
        assert np.array_equal(np.sort(got), np.sort(a))


def test_inplace_full_size_f64(hs):
    """2^27 float64 keys (the benchmark's array size) sorted in place:
    identical to numpy's sort of the same numbers (no NaNs or zeros)."""
    a = workloads.f64(1 << 27, "uniform", seed=2)
    t = _gpu(a)
    st = hs.sort_(t, opts=_ip(hs), stats=True)
    assert np.array_equal(t.cpu().numpy().view(np.uint64), np.sort(a).view(np.uint64))
    assert st["passes"] >= 14
