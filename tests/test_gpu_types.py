"""uint32 and int64 keys and the stable argsort on the GPU, against the oracle.

Bit-exact at sizes that span tiles, on-chip tasks and ragged tails; the
argsort output is unique (equal keys keep their input order), so indices
are compared exactly too.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIZES = [2, 3, 1000, 8193, 100003, (1 << 20) + 7]


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hsort


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _u32(n, seed):
    g = workloads.rng(seed)
    a = g.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    if n >= 4:
        a[:4] = [0, 2 ** 32 - 1, 2 ** 31, 2 ** 31 - 1]
    return a


def _i64(n, seed):
    g = workloads.rng(seed)
    a = g.integers(-2 ** 63, 2 ** 63 - 1, n, dtype=np.int64)
    if n >= 6:
        a[:6] = [-2 ** 63, 2 ** 63 - 1, 0, -1, 1, -2 ** 32]
    return a


@pytest.mark.parametrize("n", SIZES)
def test_sort_u32(hs, oracle_mod, n):
    a = _u32(n, n)
    t = _gpu(a)
    hs.sort_(t)
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_u32(a))


@pytest.mark.parametrize("n", SIZES)
def test_sort_i64(hs, oracle_mod, n):
    a = _i64(n, n + 1)
    t = _gpu(a)
    hs.sort_(t)
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i64(a))


def test_sort_new_types_duplicates_and_forced_levels(hs, oracle_mod):
    g = workloads.rng(5)
    n = 300007
    u = (g.integers(0, 5, n).astype(np.uint32) * np.uint32(0x3FFFFFFF))
    s = g.integers(-4, 4, n).astype(np.int64) * (2 ** 40)
    for local_T in (0, 700):
        o = hs.Opts()
        o.local_T = local_T
        t = _gpu(u)
        hs.sort_(t, opts=o)
        assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_u32(u))
        t = _gpu(s)
        hs.sort_(t, opts=o)
        assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i64(s))


@pytest.mark.parametrize("n", [1, 2, 257, 8193, 100003, (1 << 20) + 7])
def test_argsort(hs, oracle_mod, n):
    a = workloads.rng(n + 2).integers(-1000, 1000, n).astype(np.int32)
    k, idx = hs.argsort(_gpu(a))
    ok, oi = oracle_mod.argsort_i32(a)
    assert np.array_equal(k.cpu().numpy(), ok)
    assert np.array_equal(idx.cpu().numpy(), oi)


def test_argsort_in_place_and_distinct(hs, oracle_mod):
    a = workloads.uniform_i32(500001, seed=9)
    t = _gpu(a)
    idx = torch.empty_like(t)
    k, i = hs.argsort(t, out=(t, idx))
    assert k.data_ptr() == t.data_ptr()
    ok, oi = oracle_mod.argsort_i32(a)
    assert np.array_equal(t.cpu().numpy(), ok)
    assert np.array_equal(idx.cpu().numpy(), oi)


def test_new_types_learned_and_plan(hs, oracle_mod):
    a = _u32(1 << 20, 11)
    t = _gpu(a)
    st = hs.sort_(t, opts=hs.learned_opts(steps=30), stats=True)
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_u32(a))
    assert st["splitters"] > 0
    b = _i64(1 << 20, 12)
    t = _gpu(b)
    hs.sort_(t, opts=hs.learned_opts(steps=30))
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i64(b))
    # a graph-captured plan over int64 keys, replayed on fresh data
    t = torch.empty(200003, dtype=torch.int64, device="cuda")
    plan = hs.Plan(t)
    for r in range(2):
        c = _i64(t.numel(), 20 + r)
        t.copy_(_gpu(c))
        plan.run()
        plan.check()
        assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i64(c))
    plan.close()
