"""Diagnostics.  Workspace guard words (HSORT_GUARD=1): every sort path runs with 256
guard bytes after each workspace region, filled with a pattern before the
call and checked after it; none may be overwritten, and the outputs stay
bit-exact with the oracle.  HSORT_LOG=1: one line per call on stderr."""
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


@pytest.fixture
def guarded(monkeypatch):
    monkeypatch.setenv("HSORT_GUARD", "1")


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("n", [3, 1000, 5000, 300007])
def test_guards_plain_formats(hs, oracle_mod, guarded, n):
    a = workloads.uniform_i32(n, seed=n)
    t = _gpu(a)
    hs.sort_(t)
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i32(a))
    f = workloads.f64(n, "normal", seed=n)
    t = _gpu(f)
    hs.sort_(t)
    assert np.array_equal(t.cpu().numpy().view(np.uint64), oracle_mod.sort_f64(f).view(np.uint64))
    k, v = workloads.kv_dup_f64(n, seed=n, ndistinct=max(2, n // 16))
    tk, tv = _gpu(k), _gpu(v)
    hs.sort_kv_(tk, tv)
    assert np.array_equal(tk.cpu().numpy().view(np.uint64), oracle_mod.sort_kv_f64(k, v)[0].view(np.uint64))
    assert np.array_equal(k[tv.cpu().numpy()].view(np.uint64), tk.cpu().numpy().view(np.uint64))


def test_guards_in_place_learned_segmented(hs, oracle_mod, guarded):
    n = 500009
    a = workloads.uniform_i32(n, seed=1)
    o = hs.Opts()
    o.inplace = 1
    o.local_T = 900
    t = _gpu(a)
    hs.sort_(t, opts=o)
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i32(a))
    g = workloads.f64(1 << 20, "lognormal", seed=2)
    t = _gpu(g)
    hs.sort_(t, opts=hs.learned_opts(steps=20))
    assert np.array_equal(t.cpu().numpy().view(np.uint64), oracle_mod.sort_f64(g).view(np.uint64))
    off = workloads.segment_offsets(2000, 16, 1 << 14, seed=3).astype(np.int64)
    keys = workloads.uniform_i32(int(off[-1]), seed=4)
    t = _gpu(keys)
    hs.sort_segmented_(t, _gpu(off))
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_segmented_i32(keys, off))


def test_log_line(hs, monkeypatch, capfd):
    """HSORT_LOG=1: one line per sort call on stderr, with the statistics
    when they were asked for."""
    monkeypatch.setenv("HSORT_LOG", "1")
    t = _gpu(workloads.uniform_i32(100003, seed=5))
    hs.sort_(t, stats=True)
    torch.cuda.synchronize()
    err = capfd.readouterr().err
    lines = [l for l in err.splitlines() if l.startswith("[hsort]")]
    assert len(lines) == 1
    assert "op=0 n=100003" in lines[0] and "rc=0" in lines[0] and "levels=" in lines[0]
