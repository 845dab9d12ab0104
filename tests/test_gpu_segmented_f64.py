"""Batched (segmented) sorts of float64 keys on the GPU, bit-exact with the
oracle: eager calls (both level drivers), a graph-captured plan replayed on
fresh data, and the autotuner."""
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


def _keys(n, seed):
    k = workloads.f64(n, "normal", seed=seed)
    k[::11] = workloads.f64_specials()[seed % 14]  # NaNs, infinities, signed zeros among them
    return k


@pytest.mark.parametrize("lo, hi, nseg", [(1, 64, 5000), (16, 1 << 13, 3000), (16, 1 << 17, 60)])
@pytest.mark.parametrize("driver", [1, 2], ids=["host", "persistent"])
def test_segmented_f64(hs, oracle_mod, lo, hi, nseg, driver):
    off = workloads.segment_offsets(nseg, lo, hi, seed=nseg).astype(np.int64)
    keys = _keys(int(off[-1]), nseg)
    o = hs.Opts()
    o.driver = driver
    t = _gpu(keys)
    hs.sort_segmented_(t, _gpu(off), opts=o)
    assert np.array_equal(t.cpu().numpy().view(np.uint64), oracle_mod.sort_segmented_f64(keys, off).view(np.uint64))


def test_segmented_f64_plan_and_autotune(hs, oracle_mod):
    off = workloads.segment_offsets(4000, 16, 1 << 14, seed=9).astype(np.int64)
    n = int(off[-1])
    d_off = _gpu(off)
    t = torch.empty(n, dtype=torch.float64, device="cuda")
    base = hs.Opts()
    base.driver = hs.DRIVER_PERSISTENT  # the driver a plan captures
    best, rep = hs.autotune(_gpu(_keys(n, 8)), offsets=d_off, opts=base)
    assert rep["outputs_equal"] == 1
    plan = hs.Plan(t, offsets=d_off, opts=best)
    for r in range(3):
        keys = _keys(n, 10 + r)
        t.copy_(_gpu(keys))
        plan.run()
        torch.cuda.synchronize()
        plan.check()
        assert np.array_equal(t.cpu().numpy().view(np.uint64),
                              oracle_mod.sort_segmented_f64(keys, off).view(np.uint64))
    plan.close()
