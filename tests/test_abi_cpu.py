"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the header declares, and rejects bad arguments with the
documented status codes before any launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsort.h")


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    if not os.path.exists(hsort.LIB_PATH):
        from paper_1704_08579_amd import build
        build.build()
    hsort.lib()
    return hsort


def _declared():
    src = open(HEADER).read()
    return re.findall(r"HS_API\s+[\w\s\*]*?\b(hs_\w+)\s*\(", src)


def test_header_declares_entry_points():
    names = set(_declared())
    for n in ["hs_sort_i32", "hs_sort_f64", "hs_sort_kv_i32", "hs_partition_i32", "hs_sort_segmented_i32",
              "hs_workspace_size", "hs_last_error", "hs_version"]:
        assert n in names


def test_library_exports_every_declared_symbol(hs):
    L = hs.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_version(hs):
    assert hs.lib().hs_version() >= 100


def _last(hs):
    return hs.lib().hs_last_error().decode()


def test_argument_errors_before_launch(hs):
    L = hs.lib()
    assert L.hs_sort_i32(None, 5, None, None, None) == -1
    assert "NULL" in _last(hs)
    assert L.hs_sort_i32(None, -1, None, None, None) == -1
    assert L.hs_sort_i32(ctypes.c_void_p(0x1000), 1 << 31, None, None, None) == -1
    assert L.hs_sort_f64(None, 3, None, None, None) == -1
    assert L.hs_sort_kv_i32(ctypes.c_void_p(0x1000), None, 3, None, None, None) == -1
    # overlapping key and value arrays
    assert L.hs_sort_kv_i32(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1004), 3, None, None, None) == -1
    assert "overlap" in _last(hs)
    assert L.hs_partition_i32(ctypes.c_void_p(0x1000), 3, 0, None, None, None) == -1
    assert L.hs_sort_segmented_i32(ctypes.c_void_p(0x1000), 10, None, 2, None, None, None) == -1
    assert L.hs_sort_segmented_i32(ctypes.c_void_p(0x1000), 10, ctypes.c_void_p(0x2000), -1, None, None,
                                   None) == -1


def test_trivial_sizes_need_no_device(hs):
    L = hs.lib()
    st = hs.Stats()
    assert L.hs_sort_i32(None, 0, None, ctypes.addressof(st), None) == 0
    assert L.hs_sort_i32(ctypes.c_void_p(0x1000), 1, None, None, None) == 0
    assert L.hs_sort_f64(ctypes.c_void_p(0x1000), 1, None, None, None) == 0
    assert L.hs_sort_kv_i32(None, None, 0, None, None, None) == 0
    assert L.hs_sort_segmented_i32(None, 0, None, 0, None, None, None) == 0
    assert st.passes == 0 and st.bytes_alg == 0


def test_workspace_size(hs):
    n = 1 << 20
    i32 = hs.workspace_size(hs.OP_SORT_I32, n)
    f64 = hs.workspace_size(hs.OP_SORT_F64, n)
    kv = hs.workspace_size(hs.OP_SORT_KV_I32, n)
    part = hs.workspace_size(hs.OP_PARTITION_I32, n)
    seg = hs.workspace_size(hs.OP_SORT_SEGMENTED_I32, n, 1000)
    assert i32 >= 4 * n and f64 >= 8 * n and kv >= 16 * n and part >= 4 * n and seg >= i32
    assert f64 > i32 and kv > f64
    with pytest.raises(hs.HSortError):
        hs.workspace_size(99, n)
    with pytest.raises(hs.HSortError):
        hs.workspace_size(hs.OP_SORT_I32, -5)


def test_binding_rejects_cpu_tensors(hs):
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        hs.sort_(torch.zeros(4, dtype=torch.int32))
    with pytest.raises(TypeError):
        hs.sort_(torch.zeros(4, dtype=torch.int16))


def test_product_path_never_imports_oracle():
    """The package and its sources name no oracle module."""
    pkg = os.path.join(ROOT, "paper_1704_08579_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "liboracle" not in txt, f


def test_header_declares_learned_entry_points():
    names = set(_declared())
    for n in ["hs_mlp_forward_f32", "hs_mlp_grad_f32", "hs_mlp_train_f32", "hs_multiway_partition_f64"]:
        assert n in names


def test_learned_options_validated(hs):
    n = 1 << 20
    plain = hs.workspace_size(hs.OP_SORT_F64, n)
    learned = hs.workspace_size(hs.OP_SORT_F64, n, opts=hs.learned_opts())
    # sample, nested sample workspace, model, partial gradients, histograms
    assert learned > plain + (1 << 16) * 8
    # the segmented sort ignores the learned method
    seg = hs.workspace_size(hs.OP_SORT_SEGMENTED_I32, n, 10)
    assert hs.workspace_size(hs.OP_SORT_SEGMENTED_I32, n, 10, opts=hs.learned_opts()) == seg
    for bad in (hs.learned_opts(sample_log2=5), hs.learned_opts(sample_log2=21),
                hs.learned_opts(flags=hs.LEARN_FORCE_MODEL | hs.LEARN_FORCE_SAMPLE), hs.learned_opts(flags=8),
                hs.learned_opts(steps=-1), hs.learned_opts(lr=2.0)):
        with pytest.raises(hs.HSortError):
            hs.workspace_size(hs.OP_SORT_F64, n, opts=bad)
    o = hs.Opts()
    o.method = 7
    with pytest.raises(hs.HSortError):
        hs.workspace_size(hs.OP_SORT_F64, n, opts=o)


def test_learned_argument_errors_before_launch(hs):
    L = hs.lib()
    p = ctypes.c_void_p(0x1000)
    assert L.hs_mlp_forward_f32(None, None, 0, None, None) == 0
    assert L.hs_mlp_forward_f32(None, p, 5, p, None) == -1
    assert L.hs_mlp_grad_f32(p, p, p, 0, p, None) == -1
    assert L.hs_mlp_grad_f32(p, p, p, (1 << 20) + 1, p, None) == -1
    assert L.hs_mlp_grad_f32(None, p, p, 10, p, None) == -1
    assert L.hs_mlp_train_f32(p, p, 10, -1, 0.01, 0, p, None, None) == -1
    assert L.hs_mlp_train_f32(p, p, 10, 5, 0.0, 0, p, None, None) == -1
    assert L.hs_mlp_train_f32(p, p, 10, 5, 0.01, 0, None, None, None) == -1
    assert L.hs_multiway_partition_f64(p, 10, p, 256, p, None) == -1
    assert L.hs_multiway_partition_f64(p, 10, p, -1, p, None) == -1
    assert L.hs_multiway_partition_f64(p, 10, None, 3, p, None) == -1
    assert L.hs_multiway_partition_f64(p, 10, p, 3, None, None) == -1


def test_header_declares_plan_entry_points():
    names = set(_declared())
    for n in ["hs_plan_create", "hs_plan_exec", "hs_plan_check", "hs_plan_destroy", "hs_autotune"]:
        assert n in names


def test_plan_argument_errors_before_launch(hs):
    L = hs.lib()
    p = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p()
    assert L.hs_plan_create(hs.OP_SORT_I32, 10, 0, None, None) == -1
    assert L.hs_plan_create(hs.OP_PARTITION_I32, 10, 0, None, ctypes.byref(out)) == -1
    assert L.hs_plan_create(99, 10, 0, None, ctypes.byref(out)) == -1
    assert L.hs_plan_create(hs.OP_SORT_I32, -1, 0, None, ctypes.byref(out)) == -1
    assert L.hs_plan_create(hs.OP_SORT_I32, 1 << 31, 0, None, ctypes.byref(out)) == -1
    assert L.hs_plan_create(hs.OP_SORT_SEGMENTED_I32, 10, -1, None, ctypes.byref(out)) == -1
    o = hs.Opts()
    o.driver = hs.DRIVER_HOST
    assert L.hs_plan_create(hs.OP_SORT_I32, 10, 0, ctypes.byref(o), ctypes.byref(out)) == -1
    o = hs.Opts()
    o.leaf = 100
    assert L.hs_plan_create(hs.OP_SORT_I32, 10, 0, ctypes.byref(o), ctypes.byref(out)) == -1
    o.leaf = 2048
    assert L.hs_plan_create(hs.OP_SORT_I32, 10, 0, ctypes.byref(o), ctypes.byref(out)) == -1
    o = hs.Opts()
    o.workspace = 0x1000
    o.workspace_bytes = 1 << 20
    assert L.hs_plan_create(hs.OP_SORT_I32, 10, 0, ctypes.byref(o), ctypes.byref(out)) == -1
    assert "workspace" in _last(hs)
    assert L.hs_plan_exec(None, p, None, None, None) == -1
    assert L.hs_plan_check(None, None) == -1
    L.hs_plan_destroy(None)
    assert L.hs_autotune(hs.OP_SORT_I32, p, None, 10, None, 0, None, None, None, None) == -1
    best = hs.Opts()
    assert L.hs_autotune(99, p, None, 10, None, 0, None, ctypes.byref(best), None, None) == -1


def test_noalloc_rejects_sizes_beyond_its_scratch(hs):
    """hs_sort_i32_noalloc checks n against its static scratch before it
    touches a device."""
    L = hs.lib()
    assert L.hs_sort_i32_noalloc(ctypes.c_void_p(0x1000), (1 << 22) + 1, None) == -1
    assert "static scratch" in _last(hs)
    assert L.hs_sort_i32_noalloc(None, 5, None) == -1
    assert L.hs_sort_i32_noalloc(ctypes.c_void_p(0x1000), -1, None) == -1
