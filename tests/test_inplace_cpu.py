"""In-place partition levels: the option's argument checks and workspace
sizes, on the CPU (no device work: every refusal happens before a launch)."""
import ctypes

import pytest


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    return hsort


def _ip(hs, **kw):
    o = hs.Opts()
    o.inplace = 1
    for k, v in kw.items():
        setattr(o, k, v)
    return o


@pytest.mark.parametrize("op, word", [("OP_SORT_I32", 4), ("OP_SORT_F64", 8), ("OP_SORT_KV_I32", 8),
                                      ("OP_SORT_KV_F64", 16), ("OP_SORT_U32", 4), ("OP_SORT_I64", 8)])
def test_inplace_workspace_holds_no_copy_of_the_keys(hs, op, word):
    n = 1 << 24
    code = getattr(hs, op)
    out_of_place = hs.workspace_size(code, n)
    in_place = hs.workspace_size(code, n, opts=_ip(hs))
    # the buffer of order words is gone; what replaces it is one bit per key
    # and 4 bytes per 64-key row, for every tile a level can have (partial
    # tiles at segment ends included), next to the lists both modes share
    assert out_of_place - in_place >= 0.7 * word * n
    assert n // 8 <= in_place < 2.5 * n


def test_inplace_partition_workspace(hs):
    n = 1 << 24
    assert hs.workspace_size(hs.OP_PARTITION_I32, n) >= 4 * n
    assert hs.workspace_size(hs.OP_PARTITION_I32, n, opts=_ip(hs)) < n // 4  # bits + row prefixes


def test_inplace_refusals(hs):
    """Options are checked with the rest of the call's arguments (the sort
    entry points check them when they size their workspace, which
    hs_workspace_size does without a device)."""
    L = hs.lib()
    p = ctypes.c_void_p
    bad = hs.Opts()
    bad.inplace = 2
    for o, what in ((bad, "inplace"), (_ip(hs, method=hs.METHOD_LEARNED), "learned"),
                    (_ip(hs, driver=hs.DRIVER_PERSISTENT), "persistent"), (_ip(hs, autotune=1), "autotune")):
        with pytest.raises(hs.HSortError, match=what):
            hs.workspace_size(hs.OP_SORT_F64, 1 << 20, opts=o)
    plan = p()
    assert L.hs_plan_create(hs.OP_SORT_I32, 1 << 20, 0, ctypes.byref(_ip(hs)), ctypes.byref(plan)) == -1
    assert "graph" in L.hs_last_error().decode()
    best, rep = hs.Opts(), hs.TuneReport()
    assert L.hs_autotune(hs.OP_SORT_I32, p(0x1000), None, 1 << 20, None, 0, ctypes.byref(_ip(hs)),
                         ctypes.byref(best), ctypes.byref(rep), None) == -1


def test_guard_words_enlarge_the_workspace(hs, monkeypatch):
    """HSORT_GUARD=1 adds 256 guard bytes after every workspace region."""
    n = 1 << 20
    plain = hs.workspace_size(hs.OP_SORT_F64, n)
    monkeypatch.setenv("HSORT_GUARD", "1")
    guarded = hs.workspace_size(hs.OP_SORT_F64, n)
    assert guarded >= plain + 8 * 256
    monkeypatch.setenv("HSORT_GUARD", "0")
    assert hs.workspace_size(hs.OP_SORT_F64, n) == plain
