"""The on-chip tier through the C ABI, against the oracle.

* single tasks at the sizes where the on-chip sort changes regime: one
  wave's network (512 / 1024 keys: by default a whole array of up to 1024
  keys is a single wave's network, leaf=512 routes it through the workgroup
  instead), one wave's span (1024 keys), a few spans, the on-chip limit
  (8192 keys);
* an input built by McIlroy's adversary for the block levels run with the
  paper's 3-value pivot (tests/helpers.py): thousands of block levels inside
  one task, each queueing a small child, so the wave queue fills and is
  drained between block levels; int32, float64 and key/value words, alone
  and as segments of a batched sort.
"""
import numpy as np
import pytest

import workloads
from helpers import kv_index_check, median3_adversary

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

THRESHOLDS = [513, 600, 1000, 1023, 1024, 1025, 1100, 2047, 2048, 2049, 4095, 4097, 8191, 8192]


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hsort


@pytest.fixture(scope="module")
def adv():
    return median3_adversary(8192)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _sort(hs, a, opts=None):
    t = _gpu(a)
    hs.sort_(t, opts=opts)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _sort_kv(hs, k, v, opts=None):
    tk, tv = _gpu(k), _gpu(v)
    hs.sort_kv_(tk, tv, opts=opts)
    torch.cuda.synchronize()
    return tk.cpu().numpy(), tv.cpu().numpy()


@pytest.mark.parametrize("leaf", [0, 512], ids=["default", "leaf512"])
@pytest.mark.parametrize("n", THRESHOLDS)
def test_task_sizes(hs, oracle_mod, n, leaf):
    """Up to 1024 keys a whole array is one wave's network by default;
    leaf=512 sends 513..1024 keys through the on-chip workgroup instead."""
    o = hs.Opts()
    o.leaf = leaf
    a = workloads.uniform_i32(n, seed=n)
    assert np.array_equal(_sort(hs, a, o), oracle_mod.sort_i32(a))
    f = workloads.f64(n, "normal", seed=n + 1)
    assert np.array_equal(_sort(hs, f, o).view(np.uint64), oracle_mod.sort_f64(f).view(np.uint64))
    k, v = workloads.kv_dup_i32(n, seed=n + 2, ndistinct=max(2, n // 8))
    ko, vo = _sort_kv(hs, k, v, o)
    assert np.array_equal(ko, oracle_mod.sort_kv_i32(k, v)[0])
    kv_index_check(k, ko, vo)


def test_adversary_forces_levels(adv):
    """CPU check of the input itself: a permutation of 0..8191 whose first
    sampled keys are small (the adversary's doing), not sorted."""
    assert np.array_equal(np.sort(adv), np.arange(8192, dtype=np.int32))
    assert adv[0] < 16 and adv[8191] < 16
    assert not np.all(adv[:-1] <= adv[1:])


@pytest.mark.parametrize("pivot", [0, 1, 2, 3])
def test_queue_drains_i32(hs, oracle_mod, adv, pivot):
    o = hs.Opts()
    o.pivot_rule = pivot
    assert np.array_equal(_sort(hs, adv, o), oracle_mod.sort_i32(adv))
    neg = (adv.astype(np.int64) * 524287 - 2 ** 31 + 1).astype(np.int32)  # same order, spread over the range
    assert np.array_equal(_sort(hs, neg, o), oracle_mod.sort_i32(neg))


def test_adversary_reaches_deep_levels(hs, adv):
    """With the 3-value pivot, the adversarial task's on-chip phase runs
    thousands of block levels where a random task of the same size runs
    about four: it takes far longer (a witness that the queue-draining path
    ran, not a timing bar)."""
    o = hs.Opts()
    o.pivot_rule = 1
    rnd = workloads.uniform_i32(adv.size, seed=9)
    for _ in range(2):  # warm
        hs.sort_(_gpu(rnd), opts=o)
    t_adv = min(hs.sort_(_gpu(adv), opts=o, stats=True)["local_ms"] for _ in range(3))
    t_rnd = min(hs.sort_(_gpu(rnd), opts=o, stats=True)["local_ms"] for _ in range(3))
    assert t_adv > 20 * t_rnd, (t_adv, t_rnd)


@pytest.mark.parametrize("pivot", [0, 1])
def test_queue_drains_f64_and_kv(hs, oracle_mod, adv, pivot):
    o = hs.Opts()
    o.pivot_rule = pivot
    f = adv.astype(np.float64) * -0.25  # reversed order, negative values and a signed zero
    assert np.array_equal(_sort(hs, f, o).view(np.uint64), oracle_mod.sort_f64(f).view(np.uint64))
    g = adv.astype(np.float64) * 0.25 - 1000.0  # the adversary's order, negative and positive values
    assert np.array_equal(_sort(hs, g, o).view(np.uint64), oracle_mod.sort_f64(g).view(np.uint64))
    v = np.arange(adv.size, dtype=np.int32)
    ko, vo = _sort_kv(hs, adv, v, o)
    assert np.array_equal(ko, oracle_mod.sort_kv_i32(adv, v)[0])
    kv_index_check(adv, ko, vo)


@pytest.mark.parametrize("pivot", [0, 1])
def test_queue_drains_segmented(hs, oracle_mod, adv, pivot):
    """20 adversarial tasks among 40 random segments in one batched sort."""
    o = hs.Opts()
    o.pivot_rule = pivot
    g = workloads.rng(77)
    parts, off = [], [0]
    for i in range(60):
        p = adv if i % 3 == 0 else workloads.uniform_i32(int(g.integers(1, 8193)), seed=100 + i)
        parts.append(p)
        off.append(off[-1] + p.size)
    keys = np.concatenate(parts)
    off = np.asarray(off, dtype=np.int64)
    t = _gpu(keys)
    hs.sort_segmented_(t, _gpu(off), opts=o)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_segmented_i32(keys, off))


@pytest.mark.parametrize("sizes", ["all16", "all32", "mixed40", "mixed16", "ragged"])
def test_batched_tiny_arrays(hs, oracle_mod, sizes):
    """Batches of tiny arrays: groups of four tasks that all fit 16 (32) keys
    are sorted by one wave four (two) at a time; mixed groups one by one."""
    g = workloads.rng(hash(sizes) & 0xFFFF)
    n = {"all16": 40000, "all32": 30000, "mixed40": 50001, "mixed16": 40003, "ragged": 4001}[sizes]
    if sizes == "all16":
        s = np.full(n, 16)
    elif sizes == "all32":
        s = np.full(n, 32)
    elif sizes == "mixed40":
        s = g.integers(1, 41, n)
    elif sizes == "mixed16":
        s = g.integers(0, 17, n)
    else:  # a group count that is not a multiple of four, sizes at the packing bounds
        s = g.choice(np.array([15, 16, 17, 31, 32, 33]), n)
    off = np.concatenate([[0], np.cumsum(s)]).astype(np.int64)
    keys = workloads.uniform_i32(int(off[-1]), seed=n)
    keys[::7] = keys[0]  # duplicates inside the arrays
    t = _gpu(keys)
    hs.sort_segmented_(t, _gpu(off))
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_segmented_i32(keys, off))
