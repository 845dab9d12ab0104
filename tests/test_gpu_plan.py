"""Graph plans (hs_plan_*) and the autotuner, through the C ABI.

A plan records a sort of a fixed shape into a HIP graph (on the buffers of
its first replay, recorded again when a replay names other buffers); every
test replays it several times with fresh data, with eager work of the program's
own (copies and an unrelated sort) and synchronizations between the
replays, and checks every replay against the oracle.  The autotuner must
leave its input unchanged, find every candidate's output identical, and
hand back knobs from its candidate set.
"""
import numpy as np
import pytest

import workloads
from helpers import kv_index_check

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


def _eager_noise(hs, seed):
    """Unrelated eager work between replays."""
    x = _gpu(workloads.uniform_i32(100003, seed=seed))
    hs.sort_(x)
    torch.cuda.synchronize()
    assert bool((x[1:] >= x[:-1]).all())


def test_plan_segmented_replays(hs, oracle_mod):
    off = workloads.segment_offsets(3000, 16, 1 << 16, seed=41)
    off = off.astype(np.int64)
    n = int(off[-1])
    t = torch.empty(n, dtype=torch.int32, device="cuda")
    o = _gpu(off)
    plan = hs.Plan(t, offsets=o)
    for r in range(3):
        keys = workloads.uniform_i32(n, seed=42 + r)
        t.copy_(_gpu(keys))
        torch.cuda.synchronize()
        plan.run()
        plan.check()
        assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_segmented_i32(keys, off)), r
        _eager_noise(hs, r)
    plan.close()


@pytest.mark.parametrize("dist", ["uniform", "lognormal"])
def test_plan_f64_replays(hs, oracle_mod, dist):
    n = (1 << 20) + 321
    t = torch.empty(n, dtype=torch.float64, device="cuda")
    plan = hs.Plan(t)
    for r in range(3):
        x = workloads.f64(n, dist, seed=50 + r)
        t.copy_(_gpu(x))
        plan.run()
        plan.check()
        assert np.array_equal(t.cpu().numpy().view(np.uint64), oracle_mod.sort_f64(x).view(np.uint64)), r
        _eager_noise(hs, 10 + r)


def test_plan_kv_replays(hs, oracle_mod):
    n = 700001
    k = torch.empty(n, dtype=torch.int32, device="cuda")
    v = torch.empty(n, dtype=torch.int32, device="cuda")
    plan = hs.Plan(k, vals=v)
    for r in range(2):
        keys, vals = workloads.kv_dup_i32(n, seed=60 + r, ndistinct=5000)
        k.copy_(_gpu(keys))
        v.copy_(_gpu(vals))
        plan.run()
        plan.check()
        ko, vo = k.cpu().numpy(), v.cpu().numpy()
        ok, _ = oracle_mod.sort_kv_i32(keys, vals)
        assert np.array_equal(ko, ok)
        kv_index_check(keys, ko, vo)
        _eager_noise(hs, 20 + r)


def test_plan_learned(hs, oracle_mod):
    n = 1 << 20
    t = torch.empty(n, dtype=torch.float64, device="cuda")
    plan = hs.Plan(t, opts=hs.learned_opts(steps=50))
    for r in range(2):
        x = workloads.f64(n, "mixture", seed=70 + r)
        t.copy_(_gpu(x))
        plan.run()
        plan.check()
        assert np.array_equal(t.cpu().numpy().view(np.uint64), oracle_mod.sort_f64(x).view(np.uint64)), r


@pytest.mark.parametrize("kind", ["i32", "f64", "kv", "seg"])
def test_plan_on_other_buffers(hs, oracle_mod, kind):
    """One plan sorts several tensor sets of its shape: A, B, A again (each
    change of buffers records the graph again and updates it in place),
    every replay bit-exact against the oracle."""
    n = 300007
    off = workloads.segment_offsets(400, 16, 1 << 12, seed=95).astype(np.int64) if kind == "seg" else None
    if off is not None:
        n = int(off[-1])
    sets = []
    for r in range(2):
        if kind == "f64":
            sets.append((torch.empty(n, dtype=torch.float64, device="cuda"), None))
        else:
            sets.append((torch.empty(n, dtype=torch.int32, device="cuda"),
                         torch.empty(n, dtype=torch.int32, device="cuda") if kind == "kv" else None))
    o = _gpu(off) if off is not None else None
    o2 = o.clone() if o is not None else None
    plan = hs.Plan(sets[0][0], vals=sets[0][1], offsets=o)
    for r, which in enumerate([0, 1, 1, 0]):
        k, v = sets[which]
        if kind == "f64":
            x = workloads.f64(n, "normal", seed=96 + r)
        elif kind == "kv":
            x, vals = workloads.kv_dup_i32(n, seed=96 + r, ndistinct=3000)
            v.copy_(_gpu(vals))
        else:
            x = workloads.uniform_i32(n, seed=96 + r)
        k.copy_(_gpu(x))
        plan.run(k, vals=v, offsets=(o if which == 0 else o2))
        plan.check()
        got = k.cpu().numpy()
        if kind == "f64":
            assert np.array_equal(got.view(np.uint64), oracle_mod.sort_f64(x).view(np.uint64)), r
        elif kind == "kv":
            assert np.array_equal(got, oracle_mod.sort_kv_i32(x, vals)[0]), r
            kv_index_check(x, got, v.cpu().numpy())
        elif kind == "seg":
            assert np.array_equal(got, oracle_mod.sort_segmented_i32(x, off)), r
        else:
            assert np.array_equal(got, oracle_mod.sort_i32(x)), r
    with pytest.raises(ValueError):
        plan.run(torch.empty(n + 1, dtype=sets[0][0].dtype, device="cuda"))
    plan.close()


def test_plan_rejects_host_driver(hs):
    t = torch.empty(1000, dtype=torch.int32, device="cuda")
    o = hs.Opts()
    o.driver = hs.DRIVER_HOST
    with pytest.raises(hs.HSortError):
        hs.Plan(t, opts=o)


def test_autotune_segmented(hs, oracle_mod):
    off = workloads.segment_offsets(2000, 16, 1 << 15, seed=80).astype(np.int64)
    n = int(off[-1])
    keys = workloads.uniform_i32(n, seed=81)
    t, o = _gpu(keys), _gpu(off)
    base = hs.Opts()
    base.driver = hs.DRIVER_PERSISTENT
    best, rep = hs.autotune(t, offsets=o, opts=base)
    assert rep["candidates"] == 18 and rep["outputs_equal"] == 1
    assert rep["best_ms"] <= rep["default_ms"]
    assert best.local_T in (2048, 4096, 8192) and best.leaf in (256, 512, 1024) and best.pivot_rule in (2, 3)
    assert np.array_equal(t.cpu().numpy(), keys), "the autotuner changed its input"
    best2, rep2 = hs.autotune(t, offsets=o, opts=base)
    assert rep2["candidates"] == 0
    assert (best2.local_T, best2.leaf, best2.pivot_rule) == (best.local_T, best.leaf, best.pivot_rule)
    plan = hs.Plan(t, offsets=o, opts=best)
    plan.run()
    plan.check()
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_segmented_i32(keys, off))


def test_autotune_flag(hs, oracle_mod):
    """opts.autotune: the first call tunes, later calls of the size class reuse it."""
    a = workloads.uniform_i32(300007, seed=90)
    o = hs.Opts()
    o.autotune = 1
    for r in range(2):
        t = _gpu(a)
        hs.sort_(t, opts=o)
        assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i32(a))
    off = workloads.segment_offsets(500, 16, 1 << 14, seed=91).astype(np.int64)
    keys = workloads.uniform_i32(int(off[-1]), seed=92)
    t, ot = _gpu(keys), _gpu(off)
    plan = hs.Plan(t, offsets=ot, opts=o)
    plan.run()
    plan.check()
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_segmented_i32(keys, off))


def test_plan_persistent_tail(hs, oracle_mod):
    """Skewed splits (median-of-3 on an organ pipe, small on-chip limit) need
    more levels than the plan records as per-level launches; the persistent
    driver recorded after them finishes the sort."""
    n = 400003
    half = np.arange(n // 2, dtype=np.int32)
    base = np.concatenate([half, half[::-1], [7]]).astype(np.int32)
    o = hs.Opts()
    o.pivot_rule = 1
    o.local_T = 600
    t = torch.empty(n, dtype=torch.int32, device="cuda")
    plan = hs.Plan(t, opts=o)
    for r in range(2):
        x = np.roll(base, 1000 * r)
        t.copy_(_gpu(x))
        plan.run()
        plan.check()
        assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i32(x)), r
    st = hs.sort_(_gpu(base), opts=o, stats=True)
    assert st["passes"] > 12  # more than the 11 + 1 levels the plan records


# ------------------------------------------------------------- full sizes (properties)

def _segment_checks(keys_in, keys_out, off):
    """Every segment sorted, and a permutation of its input (per-segment sums
    of two mixing functions of the keys)."""
    seg_start = off[:-1]
    nonempty = off[1:] > off[:-1]
    d = np.diff(keys_out.astype(np.int64))
    boundary = np.zeros(keys_out.size, dtype=bool)
    boundary[off[1:-1]] = True
    assert np.all((d >= 0) | boundary[1:]), "a segment is not sorted"
    u_in = keys_in.astype(np.uint32).astype(np.uint64)
    u_out = keys_out.astype(np.uint32).astype(np.uint64)
    for mix in (lambda u: (u * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF),
                lambda u: (u ^ (u >> np.uint64(7))) * (u | np.uint64(1)) & np.uint64(0xFFFFFFFFFF)):
        a = np.add.reduceat(mix(u_in), seg_start[nonempty])
        b = np.add.reduceat(mix(u_out), seg_start[nonempty])
        assert np.array_equal(a, b), "a segment is not a permutation of its input"


@pytest.mark.parametrize("name,nseg,lo,hi", [("A", 200000, 16, 1 << 13), ("B", 2840, 16, 1 << 20)])
def test_full_size_batched_graph(hs, name, nseg, lo, hi):
    """The batched workloads bench.py times (one autotuned graph replay)."""
    off = workloads.segment_offsets(nseg, lo, hi, seed=5).astype(np.int64)
    keys = workloads.uniform_i32(int(off[-1]), seed=6)
    t, o = _gpu(keys), _gpu(off)
    base = hs.Opts()
    base.driver = hs.DRIVER_PERSISTENT
    tuned, _ = hs.autotune(t, offsets=o, opts=base)
    plan = hs.Plan(t, offsets=o, opts=tuned)
    plan.run()
    plan.check()
    _segment_checks(keys, t.cpu().numpy(), off)
    plan.close()


def test_full_size_learned(hs):
    """2^28 float64 lognormal keys with learned splitters (the size bench.py
    times): sorted by totalOrder and a permutation of the input."""
    x = workloads.f64(1 << 28, "lognormal", seed=6)
    t = _gpu(x)
    st = hs.sort_(t, opts=hs.learned_opts(seed=100), stats=True)
    got = t.cpu().numpy().view(np.uint64)
    del t
    assert st["splitters"] > 0
    assert np.array_equal(np.sort(x).view(np.uint64), got)
