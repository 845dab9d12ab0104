"""The largest array the C ABI accepts: n = 2^31 - 1 keys (int32: 8 GiB, float64: 16 GiB).
Positions inside the kernels are 32-bit; this runs the whole tiered path
with indices up to the limit.  The checks are properties that hold at any
size (the oracle would take minutes here): the output is non-decreasing,
and two multiset fingerprints of the keys (their sum, and the sum of a
mixing function of each key) are unchanged."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hsort


def _fingerprints(t):
    x = t if t.dtype == torch.int64 else t.to(torch.int64)
    mixed = (x * 0x9E3779B1 + 0x7F4A7C15) ^ (x >> 7)  # a different weight per key value
    return int(x.sum().item()), int(mixed.sum().item())


def test_max_size_i32(hs):
    n = (1 << 31) - 1
    g = torch.Generator(device="cuda")
    g.manual_seed(31)
    t = torch.randint(-(2 ** 31), 2 ** 31, (n,), dtype=torch.int32, device="cuda", generator=g)
    t[:1000] = 2 ** 31 - 1  # extremes at both ends of the order
    t[-1000:] = -(2 ** 31)
    before = _fingerprints(t)
    st = hs.sort_(t, stats=True)
    torch.cuda.synchronize()
    assert bool((t[1:] >= t[:-1]).all().item())
    assert _fingerprints(t) == before
    assert int(t[0].item()) == -(2 ** 31) and int(t[-1].item()) == 2 ** 31 - 1
    assert st["passes"] >= 18


def test_max_size_f64(hs):
    """2^31 - 1 float64 keys (16 GiB; 8-byte words, their own tile shapes):
    non-decreasing (no NaNs or zeros: numeric order is totalOrder) and the
    bit patterns' fingerprints unchanged."""
    n = (1 << 31) - 1
    g = torch.Generator(device="cuda")
    g.manual_seed(32)
    t = torch.randn((n,), dtype=torch.float64, device="cuda", generator=g)
    before = _fingerprints(t.view(torch.int64))
    hs.sort_(t)
    torch.cuda.synchronize()
    assert bool((t[1:] >= t[:-1]).all().item())
    assert _fingerprints(t.view(torch.int64)) == before


def test_max_size_i32_in_place(hs):
    """The in-place partition levels at the limit: their key bits, row and
    tile prefixes are indexed across 2^31 - 1 keys."""
    n = (1 << 31) - 1
    g = torch.Generator(device="cuda")
    g.manual_seed(33)
    t = torch.randint(-1000, 1000, (n,), dtype=torch.int32, device="cuda", generator=g)  # heavy duplicates
    before = _fingerprints(t)
    o = hs.Opts()
    o.inplace = 1
    hs.sort_(t, opts=o)
    torch.cuda.synchronize()
    assert bool((t[1:] >= t[:-1]).all().item())
    assert _fingerprints(t) == before
