"""Sorts on several HIP streams.  Whole arrays that are one on-chip task
return without reading anything back, so calls on two streams overlap on
the device; the library's cached workspace is shared, and an event orders
its uses.  A caller-provided workspace per stream needs no ordering."""
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


def test_two_streams_share_the_workspace(hs, oracle_mod):
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    arrays = [workloads.uniform_i32(1100 + 433 * i, seed=i) for i in range(24)]  # one on-chip task each
    arrays += [workloads.f64(600 + 251 * i, "normal", seed=i) for i in range(8)]
    ts = [_gpu(a) for a in arrays]
    torch.cuda.synchronize()
    for i, t in enumerate(ts):
        with torch.cuda.stream(streams[i % 2]):
            hs.sort_(t)
    torch.cuda.synchronize()
    for a, t in zip(arrays, ts):
        want = oracle_mod.sort_i32(a) if a.dtype == np.int32 else oracle_mod.sort_f64(a)
        assert np.array_equal(t.cpu().numpy().view(np.uint8), want.view(np.uint8))


def test_workspace_per_stream(hs, oracle_mod):
    n = 300007
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wbytes = hs.workspace_size(hs.OP_SORT_F64, n)
    arrays = [workloads.f64(n, "uniform", seed=40 + i) for i in range(2)]
    ts = [_gpu(a) for a in arrays]
    wss = [torch.empty(wbytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
    torch.cuda.synchronize()
    for s, t, ws in zip(streams, ts, wss):
        o = hs.Opts()
        o.workspace = ws.data_ptr()
        o.workspace_bytes = wbytes
        with torch.cuda.stream(s):
            hs.sort_(t, opts=o)
    torch.cuda.synchronize()
    for a, t in zip(arrays, ts):
        assert np.array_equal(t.cpu().numpy().view(np.uint64), oracle_mod.sort_f64(a).view(np.uint64))
