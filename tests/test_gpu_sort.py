"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Element-by-element comparison at sizes the oracle finishes in seconds,
spanning several partition tiles, several on-chip tasks and ragged tails;
the bar is bit-exact (integer keys, float64 bit patterns, key/value keys plus
the pair multiset).  Full-size runs are checked through properties that hold
at any size (sorted by key, permutation of the input).
"""
import numpy as np
import pytest

import workloads
from helpers import kv_index_check, pair_multiset_equal

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


def _run_i32(hs, a, opts=None):
    t = _gpu(a)
    hs.sort_(t, opts=opts)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _opts(hs, pivot=0, local_T=0):
    o = hs.Opts()
    o.pivot_rule = pivot
    o.local_T = local_T
    return o


# the last two straddle the first batch's margin change (levels_for 8 -> 9 at T = 8192)
SIZES = [2, 3, 63, 64, 65, 255, 256, 257, 1000, 4095, 4096, 4097, 8192, 8193, 16383, 16384, 16385,
         50001, (1 << 17) + 13, 1 << 20, (1 << 20) + 1]


@pytest.mark.parametrize("n", SIZES)
def test_sort_i32_sizes(hs, oracle_mod, n):
    a = workloads.uniform_i32(n, seed=100 + n)
    assert np.array_equal(_run_i32(hs, a), oracle_mod.sort_i32(a))


def test_sort_i32_config0(hs, oracle_mod):
    """2^20 uniform int32 over the full range, seed 1 (sort bound 256)."""
    a = workloads.uniform_i32(1 << 20, seed=1)
    assert np.array_equal(_run_i32(hs, a), oracle_mod.sort_i32(a))


@pytest.mark.parametrize("pivot", [1, 2, 3])
@pytest.mark.parametrize("local_T", [300, 1024, 4096])
def test_sort_i32_forced_levels(hs, oracle_mod, pivot, local_T):
    """A small on-chip limit forces many global partition levels."""
    a = workloads.uniform_i32(300001, seed=7)
    assert np.array_equal(_run_i32(hs, a, _opts(hs, pivot, local_T)), oracle_mod.sort_i32(a))


def _adversarial(n, seed):
    g = workloads.rng(seed)
    half = np.arange(n // 2, dtype=np.int32)
    return {
        "all_equal": np.full(n, 7, dtype=np.int32),
        "two_values": g.integers(0, 2, n).astype(np.int32),
        "few_values": g.integers(-3, 4, n).astype(np.int32),
        "sorted": np.sort(workloads.uniform_i32(n, seed)),
        "reverse": np.sort(workloads.uniform_i32(n, seed))[::-1].copy(),
        "organ_pipe": np.concatenate([half, half[::-1]]).astype(np.int32),
        "extremes": g.choice(np.array([-(2 ** 31), 2 ** 31 - 1, 0, -1], dtype=np.int64), n).astype(np.int32),
        "sawtooth": (np.arange(n) % 1000).astype(np.int32),
    }


@pytest.mark.parametrize("kind", ["all_equal", "two_values", "few_values", "sorted", "reverse", "organ_pipe",
                                  "extremes", "sawtooth"])
@pytest.mark.parametrize("pivot", [1, 3])
def test_sort_i32_adversarial(hs, oracle_mod, kind, pivot):
    a = _adversarial(200003, 5)[kind]
    assert np.array_equal(_run_i32(hs, a, _opts(hs, pivot, 2048)), oracle_mod.sort_i32(a))
    assert np.array_equal(_run_i32(hs, a, _opts(hs, pivot)), oracle_mod.sort_i32(a))


@pytest.mark.parametrize("dist", ["uniform", "normal", "sorted", "reverse", "lognormal", "zipf", "mixture"])
def test_sort_f64(hs, oracle_mod, dist):
    a = workloads.f64(300007, dist, seed=2)
    t = _gpu(a)
    hs.sort_(t)
    got = t.cpu().numpy()
    assert np.array_equal(got.view(np.uint64), oracle_mod.sort_f64(a).view(np.uint64))


def test_sort_f64_specials(hs, oracle_mod):
    """NaNs of both signs, infinities, signed zeros, denormals mixed in."""
    g = workloads.rng(3)
    a = workloads.f64(100000, "normal", seed=3)
    sp = workloads.f64_specials()
    a[g.integers(0, a.size, 5000)] = sp[g.integers(0, sp.size, 5000)]
    for local_T in (0, 512):
        t = _gpu(a)
        hs.sort_(t, opts=_opts(hs, 0, local_T))
        got = t.cpu().numpy()
        assert np.array_equal(got.view(np.uint64), oracle_mod.sort_f64(a).view(np.uint64))


@pytest.mark.parametrize("n", [2, 200, 256, 257, 5000, 8192, 8193, 100003])
def test_sort_kv_sizes(hs, oracle_mod, n):
    keys, vals = workloads.kv_dup_i32(n, seed=4 + n, ndistinct=max(2, n // 16), force_extremes=True)
    k, v = _gpu(keys), _gpu(vals)
    hs.sort_kv_(k, v)
    ko, vo = k.cpu().numpy(), v.cpu().numpy()
    ok, _ = oracle_mod.sort_kv_i32(keys, vals)
    assert np.array_equal(ko, ok)
    kv_index_check(keys, ko, vo)


def test_sort_kv_arbitrary_values(hs, oracle_mod):
    g = workloads.rng(31)
    keys = g.integers(-100, 100, 250000).astype(np.int32)
    vals = g.integers(-(2 ** 31), 2 ** 31, 250000, dtype=np.int32)
    vals[:1000] = -1
    keys[:1000] = 2 ** 31 - 1
    for local_T in (0, 700):
        k, v = _gpu(keys), _gpu(vals)
        hs.sort_kv_(k, v, opts=_opts(hs, 0, local_T))
        ko, vo = k.cpu().numpy(), v.cpu().numpy()
        ok, ov = oracle_mod.sort_kv_i32(keys, vals)
        assert np.array_equal(ko, ok)
        assert pair_multiset_equal(keys, vals, ko, vo)


@pytest.mark.parametrize("n", [1, 5, 4096, 4097, 100000, (1 << 20) + 3])
def test_partition(hs, oracle_mod, n):
    a = workloads.uniform_i32(n, seed=50 + n)
    g = workloads.rng(n)
    for pivot in [int(a[g.integers(0, n)]), -(2 ** 31), 2 ** 31 - 1, 0]:
        t = _gpu(a)
        cnt = hs.partition_(t, pivot)
        got = t.cpu().numpy()
        k = int(cnt.cpu().item())
        _, ok = oracle_mod.partition_le_i32(a, pivot)
        assert k == ok
        assert np.all(got[:k] <= pivot) and np.all(got[k:] > pivot)
        assert np.array_equal(np.sort(got), np.sort(a))


def test_partition_empty(hs):
    t = torch.empty(0, dtype=torch.int32, device="cuda")
    assert int(hs.partition_(t, 5).cpu().item()) == 0


@pytest.mark.parametrize("hi", [300, 20000, 100000])
def test_segmented(hs, oracle_mod, hi):
    off = workloads.segment_offsets(400, 1, hi, seed=hi)
    off = np.concatenate([[0, 0, 1], off[1:] + 1, [off[-1] + 1]]).astype(np.int64)  # empty + size-1 segments
    keys = workloads.uniform_i32(int(off[-1]), seed=hi + 1)
    t, o = _gpu(keys), _gpu(off)
    hs.sort_segmented_(t, o)
    got = t.cpu().numpy()
    assert np.array_equal(got, oracle_mod.sort_segmented_i32(keys, off))


def test_segmented_forced_levels(hs, oracle_mod):
    off = workloads.segment_offsets(50, 100, 60000, seed=3)
    keys = _adversarial(int(off[-1]), 2)["few_values"]
    t, o = _gpu(keys), _gpu(off)
    hs.sort_segmented_(t, o, opts=_opts(hs, 1, 1000))
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_segmented_i32(keys, off))


@pytest.mark.parametrize("dtype", [np.int32, np.float64])
def test_segmented_one_tile_segments(hs, oracle_mod, dtype):
    """Thousands of segments of one or two partition tiles each in one level
    list (on-chip limit 300, segments of 301-3000 keys): a workgroup's
    consecutive tiles lie hundreds of segments apart, so every tile finds its
    segment by the bounded search."""
    off = workloads.segment_offsets(6000, 301, 3000, seed=11)
    n = int(off[-1])
    keys = workloads.uniform_i32(n, seed=12) if dtype == np.int32 else workloads.f64(n, "normal", seed=12)
    t, o = _gpu(keys), _gpu(off)
    hs.sort_segmented_(t, o, opts=_opts(hs, 3, 300))
    want = oracle_mod.sort_segmented_i32(keys, off) if dtype == np.int32 else \
        oracle_mod.sort_segmented_f64(keys, off)
    assert np.array_equal(t.cpu().numpy().view(np.uint8), want.view(np.uint8))


def test_unaligned_views(hs, oracle_mod):
    """Tensors that start 4 bytes into an allocation (not 16-byte aligned)."""
    a = workloads.uniform_i32(100001, seed=77)
    base = torch.zeros(a.size + 1, dtype=torch.int32, device="cuda")
    base[1:] = _gpu(a)
    view = base[1:]
    hs.sort_(view)
    assert np.array_equal(view.cpu().numpy(), oracle_mod.sort_i32(a))


def test_stats_and_repeat(hs, oracle_mod):
    a = workloads.uniform_i32(1 << 20, seed=1)
    t = _gpu(a)
    st = hs.sort_(t, stats=True)
    n = 1 << 20
    # 2^20 keys over an on-chip limit of 2^14: at least log2(2^20 / 2^14) levels
    assert st["passes"] >= 6
    assert 6 * n <= st["keys_partitioned"] <= st["passes"] * n
    # every key is read and written once per level it takes part in, and once
    # by its on-chip sort (no equal-key fills on distinct random keys)
    assert st["bytes_alg"] == 2 * 4 * (st["keys_partitioned"] + n)
    first = t.cpu().numpy()
    t2 = _gpu(a)
    hs.sort_(t2)
    assert np.array_equal(first, t2.cpu().numpy())
    assert np.array_equal(first, oracle_mod.sort_i32(a))


# ------------------------------------------------------------- full sizes (properties)

def _f64_total_order_key(bits):
    neg = (bits >> np.uint64(63)).astype(bool)
    return np.where(neg, ~bits, bits | np.uint64(1 << 63))


@pytest.mark.parametrize("dist", ["uniform", "normal", "sorted", "reverse"])
def test_full_size_f64(hs, dist):
    """2^27 float64 keys, the size the benchmark times: sorted by key and a
    permutation of the input (compared with numpy's sort of the same bits)."""
    a = workloads.f64(1 << 27, dist, seed=2)
    t = _gpu(a)
    hs.sort_(t)
    got = t.cpu().numpy().view(np.uint64)
    k = _f64_total_order_key(got)
    assert np.all(k[:-1] <= k[1:])
    assert np.array_equal(np.sort(a).view(np.uint64), got)


@pytest.mark.parametrize("dist,seed", [("zipf", 7), ("mixture", 8)])
def test_full_size_f64_learned_inputs(hs, dist, seed):
    """2^28 float64 keys of the learned-splitter workloads (Zipf ranks with
    heavy repeats, an 8-Gaussian mixture), sorted by the plain method and by
    the learned one (which falls back to the sample's order statistics on
    these inputs): both equal numpy's sort of the same bits."""
    print(f"full size {dist} 2^28", flush=True)
    a = workloads.f64(1 << 28, dist, seed=seed)
    want = np.sort(a).view(np.uint64)  # no NaN or negative zero in these inputs
    t = _gpu(a)
    hs.sort_(t)
    assert np.array_equal(t.cpu().numpy().view(np.uint64), want), "plain"
    t.copy_(_gpu(a))
    hs.sort_(t, opts=hs.learned_opts(seed=100))
    assert np.array_equal(t.cpu().numpy().view(np.uint64), want), "learned"


def test_full_size_kv(hs):
    """2^28 int32 pairs, 2^16 distinct keys, values = index: exact index check."""
    keys, vals = workloads.kv_dup_i32(1 << 28, seed=4)
    k, v = _gpu(keys), _gpu(vals)
    hs.sort_kv_(k, v)
    ko = k.cpu().numpy()
    vo = v.cpu().numpy()
    assert np.all(ko[:-1] <= ko[1:])
    kv_index_check(keys, ko, vo)


# ------------------------------------------------------------- level drivers

def _driver_opts(hs, driver, local_T=0, pivot=0):
    o = hs.Opts()
    o.driver = driver
    o.local_T = local_T
    o.pivot_rule = pivot
    return o


@pytest.mark.parametrize("driver", [2, 1], ids=["persistent", "host"])
def test_drivers_bit_exact(hs, oracle_mod, driver):
    """Both level drivers against the oracle: many levels (small on-chip
    limit), equal-key runs, key/value pairs, f64 and segmented inputs."""
    a = workloads.uniform_i32(1 << 20, seed=1)
    t = _gpu(a)
    hs.sort_(t, opts=_driver_opts(hs, driver))
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i32(a))
    for name, x in _adversarial(300001, 9).items():
        t = _gpu(x)
        hs.sort_(t, opts=_driver_opts(hs, driver, local_T=600, pivot=1))
        assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i32(x)), name
    x = workloads.f64(700001, "normal", seed=5)
    t = _gpu(x)
    st = hs.sort_(t, opts=_driver_opts(hs, driver, local_T=1024), stats=True)
    assert np.array_equal(t.cpu().numpy().view(np.uint64), oracle_mod.sort_f64(x).view(np.uint64))
    assert st["passes"] >= 9
    # the host driver launches levels in batches (trailing empty levels included)
    assert st["partition_launches"] == 1 if driver == 2 else st["partition_launches"] >= st["passes"]
    keys, vals = workloads.kv_dup_i32(500003, seed=6, ndistinct=1000)
    k, v = _gpu(keys), _gpu(vals)
    hs.sort_kv_(k, v, opts=_driver_opts(hs, driver, local_T=2048))
    ko, vo = k.cpu().numpy(), v.cpu().numpy()
    ok, _ = oracle_mod.sort_kv_i32(keys, vals)
    assert np.array_equal(ko, ok)
    kv_index_check(keys, ko, vo)
    off = workloads.segment_offsets(300, 1, 200000, seed=8)
    keys = workloads.uniform_i32(int(off[-1]), seed=9)
    t, o = _gpu(keys), _gpu(off.astype(np.int64))
    hs.sort_segmented_(t, o, opts=_driver_opts(hs, driver, local_T=4096))
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_segmented_i32(keys, off))


def _levels_for(size, T):
    """Levels that balanced splits need to bring `size` keys down to T."""
    lv = 1
    while size > T:
        size = (size + 1) // 2
        lv += 1
    return lv


def _first_batch(size, T):
    """Levels the host-driven loop launches before its first read-back."""
    lf = _levels_for(size, T)
    return lf + (2 if lf <= 8 else 3)


def test_host_driver_levels_beyond_first_batch(hs, oracle_mod):
    """The host-driven loop runs a first batch of levels and the on-chip
    sorts before its first read-back; skewed splits (median-of-3 pivots on an
    adversarial order, a small on-chip limit) leave levels after that batch,
    which then run with the on-chip sorts a second time over the tasks they
    add.  The output must match the oracle, values riding along too."""
    n, T = 1 << 18, 600
    x = _adversarial(n, 3)["organ_pipe"]
    t = _gpu(x)
    st = hs.sort_(t, opts=_driver_opts(hs, 1, local_T=T, pivot=1), stats=True)
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i32(x))
    assert st["passes"] > _first_batch(n, T), st["passes"]
    v = np.arange(n, dtype=np.int32)
    k, vv = _gpu(x), _gpu(v)
    hs.sort_kv_(k, vv, opts=_driver_opts(hs, 1, local_T=T, pivot=1))
    ko, vo = k.cpu().numpy(), vv.cpu().numpy()
    assert np.array_equal(ko, oracle_mod.sort_kv_i32(x, v)[0])
    kv_index_check(x, ko, vo)
    f = x.astype(np.float64) * -0.5
    t = _gpu(f)
    st = hs.sort_(t, opts=_driver_opts(hs, 1, local_T=T, pivot=1), stats=True)
    assert np.array_equal(t.cpu().numpy().view(np.uint64), oracle_mod.sort_f64(f).view(np.uint64))
    assert st["passes"] > _first_batch(n, T), st["passes"]


def test_persistent_driver_barrier_timeout_is_reported(hs):
    """A grid-barrier wait capped at one poll (forced from the host) ends the
    level driver with an error instead of waiting: the call fails cleanly and
    the library keeps working."""
    x = workloads.f64(1 << 22, "uniform", seed=10)
    o = _driver_opts(hs, 2)
    o.spin_limit = 1
    failed = 0
    for _ in range(3):  # a one-poll wait fails unless every workgroup arrives at once
        t = _gpu(x)
        try:
            hs.sort_(t, opts=o)
        except hs.HSortError as e:
            assert "0x" in str(e)
            failed += 1
    assert failed >= 1
    t = _gpu(x)
    hs.sort_(t)
    assert np.array_equal(t.cpu().numpy(), np.sort(x))
