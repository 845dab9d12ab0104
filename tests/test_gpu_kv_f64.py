"""(float64 key, int32 value) pairs on the GPU, against the oracle.

The keys must equal the oracle's bit for bit and the pairs must be the
input's multiset.  Equal keys are ordered by their values' bits as unsigned
32-bit integers (the library's documented tie rule), which makes the output
unique: it is also compared exactly with a lexicographic sort of the input
pairs by (totalOrder key, value bits).  Sizes cross the one-wave network
(512 pairs), the on-chip limit (4096), several partition tiles and ragged
tails; the forced-tier cases lower the network bound and the on-chip limit
so that every tier runs on small inputs.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIZES = [2, 3, 64, 257, 512, 513, 1000, 4096, 4097, 8193, 100003, (1 << 20) + 7]


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hsort


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _input(n, seed, ndistinct=None, specials=False):
    nd = ndistinct if ndistinct is not None else max(2, min(n // 4, 1 << 16))
    keys, _ = workloads.kv_dup_f64(n, seed=seed, ndistinct=nd, specials=specials)
    vals = workloads.rng(seed + 1000).integers(-(2 ** 31), 2 ** 31, n, dtype=np.int64).astype(np.int32)
    return keys, vals


def _check(oracle_mod, keys, vals, ko, vo):
    ok, _ = oracle_mod.sort_kv_f64(keys, vals)
    assert np.array_equal(ko.view(np.uint64), ok.view(np.uint64)), "keys differ from the oracle's"
    order = np.lexsort((vals.view(np.uint32), oracle_mod.f64_order_keys(keys)))
    assert np.array_equal(ko.view(np.uint64), keys.view(np.uint64)[order])
    assert np.array_equal(vo, vals[order]), "pairs or tie order differ"


def _run(hs, keys, vals, opts=None):
    k, v = _gpu(keys), _gpu(vals)
    hs.sort_kv_(k, v, opts=opts)
    return k.cpu().numpy(), v.cpu().numpy()


@pytest.mark.parametrize("n", SIZES)
def test_kv_f64_sizes(hs, oracle_mod, n):
    keys, vals = _input(n, seed=n)
    print(f"kv_f64 n={n}", flush=True)
    _check(oracle_mod, keys, vals, *_run(hs, keys, vals))


def test_kv_f64_specials_and_few_keys(hs, oracle_mod):
    """NaNs of both signs, infinities, signed zeros and denormals among 64
    distinct keys: long runs of equal keys go through the equal-key rule."""
    for n, nd in ((300007, 64), (70001, 2)):
        keys, vals = _input(n, seed=nd, ndistinct=nd, specials=True)
        _check(oracle_mod, keys, vals, *_run(hs, keys, vals))


@pytest.mark.parametrize("knob", ["leaf64", "T700", "median3", "persistent"])
def test_kv_f64_forced_tiers(hs, oracle_mod, knob):
    o = hs.Opts()
    if knob == "leaf64":
        o.leaf = 64
    elif knob == "T700":
        o.local_T = 700
    elif knob == "median3":
        o.pivot_rule = 1
    else:
        o.driver = hs.DRIVER_PERSISTENT
    keys, vals = _input(200003, seed=7)
    _check(oracle_mod, keys, vals, *_run(hs, keys, vals, o))


def test_kv_f64_index_values_is_stable_argsort(hs):
    """Values = positions: ties by value make the sort a stable argsort of
    the float64 keys, so numpy's stable argsort decides every value."""
    n = (1 << 24) + 5
    keys, vals = workloads.kv_dup_f64(n, seed=21)
    ko, vo = _run(hs, keys, vals)
    want = np.argsort(keys, kind="stable")
    assert np.array_equal(vo, want.astype(np.int32))
    assert np.array_equal(ko.view(np.uint64), keys.view(np.uint64)[want])


def test_kv_f64_plan_and_autotune(hs, oracle_mod):
    n = 200003
    k = torch.empty(n, dtype=torch.float64, device="cuda")
    v = torch.empty(n, dtype=torch.int32, device="cuda")
    plan = hs.Plan(k, v)
    for r in range(3):
        keys, vals = _input(n, seed=30 + r)
        k.copy_(_gpu(keys))
        v.copy_(_gpu(vals))
        plan.run()
        torch.cuda.synchronize()
        plan.check()
        _check(oracle_mod, keys, vals, k.cpu().numpy(), v.cpu().numpy())
    plan.close()
    keys, vals = _input(n, seed=40)
    best, rep = hs.autotune(_gpu(keys), _gpu(vals))
    assert rep["outputs_equal"] == 1 and best.local_T <= 4096
    _check(oracle_mod, keys, vals, *_run(hs, keys, vals, best))


def test_kv_f64_full_size_properties(hs):
    """2^27 pairs (the size the benchmark times), values = positions: keys
    in totalOrder, values a permutation, every key beside its value, equal
    keys in position order."""
    n = 1 << 27
    keys, vals = workloads.kv_dup_f64(n, seed=22)
    ko, vo = _run(hs, keys, vals)
    kb = ko.view(np.uint64)
    ok = np.where(kb >> np.uint64(63) == 1, ~kb, kb | np.uint64(1 << 63))
    assert np.all(ok[:-1] <= ok[1:])
    idx = vo.astype(np.int64)
    assert np.all((idx >= 0) & (idx < n))
    assert np.bincount(idx, minlength=n).max() == 1
    assert np.array_equal(keys.view(np.uint64)[idx], kb)
    same = ok[1:] == ok[:-1]
    assert np.all(idx[1:][same] > idx[:-1][same])


@pytest.mark.parametrize("flags", [0, 1, 2], ids=["judged", "model", "sample"])
def test_kv_f64_learned(hs, oracle_mod, flags):
    """The learned front end (sample, model, 256-way pass) on float64 keys with
    values: bit-exact with the oracle whichever splitters drive the pass."""
    n = (1 << 21) + 5
    keys = np.exp(2.0 * workloads.rng(50 + flags).standard_normal(n))  # lognormal(0, 2)
    keys[:: 97] = keys[7]  # a heavy key: an equality bucket
    vals = workloads.rng(60 + flags).integers(-(2 ** 31), 2 ** 31, n, dtype=np.int64).astype(np.int32)
    k, v = _gpu(keys), _gpu(vals)
    st = hs.sort_kv_(k, v, opts=hs.learned_opts(steps=40, seed=3, flags=flags), stats=True)
    _check(oracle_mod, keys, vals, k.cpu().numpy(), v.cpu().numpy())
    assert st["splitters"] > 0
    if flags == 2:
        assert st["fallback_used"] == 1



@pytest.mark.parametrize("n", [1, 2, 513, 4097, 100003, (1 << 20) + 7])
def test_argsort_f64(hs, oracle_mod, n):
    """Stable argsort of float64 keys (specials and heavy duplicates): keys
    and positions identical to the oracle's, which are unique."""
    keys, _ = workloads.kv_dup_f64(n, seed=n + 70, ndistinct=max(2, min(n // 8, 5000)), specials=n > 100)
    ko, idx = hs.argsort(_gpu(keys))
    ok, oi = oracle_mod.argsort_f64(keys)
    assert np.array_equal(ko.cpu().numpy().view(np.uint64), ok.view(np.uint64))
    assert np.array_equal(idx.cpu().numpy(), oi)


def test_argsort_f64_in_place(hs, oracle_mod):
    keys = workloads.f64(300007, "normal", seed=71)
    keys[::3] = keys[5]
    t = _gpu(keys)
    idx = torch.empty(t.shape, dtype=torch.int32, device="cuda")
    k, i = hs.argsort(t, out=(t, idx))
    assert k.data_ptr() == t.data_ptr()
    ok, oi = oracle_mod.argsort_f64(keys)
    assert np.array_equal(t.cpu().numpy().view(np.uint64), ok.view(np.uint64))
    assert np.array_equal(idx.cpu().numpy(), oi)
