"""hsort: MI355X (gfx950) hybrid quicksort + bitonic sort.

Thin Python binding over the C ABI of ``include/hsort.h`` (libhsort.so, built
from ``csrc/`` with hipcc).  PyTorch supplies device memory and the current
HIP stream; every step of the sort runs in the library's HIP kernels.  There
is no fallback: if the library is missing or the device is not gfx950 the
calls raise.

    import torch, paper_1704_08579_amd as hsort
    x = torch.randint(-2**31, 2**31, (1 << 20,), dtype=torch.int32, device="cuda")
    hsort.sort_(x)                      # in place, ascending
    hsort.sort_kv_(keys, vals)          # values follow their keys (int32 or float64 keys)
    k = hsort.partition_(x, pivot)      # x[:k] <= pivot < x[k:]
    hsort.sort_segmented_(x, offsets)   # each [off[i], off[i+1]) on its own
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["sort_", "sort_kv_", "argsort", "partition_", "sort_segmented_", "workspace_size", "Stats", "Opts",
           "learned_opts", "mlp_forward", "mlp_grad", "mlp_train", "multiway_partition_", "learn_debug", "Plan",
           "autotune", "TuneReport", "lib", "LIB_PATH", "HSortError"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhsort.so")

HS_OK = 0
(OP_SORT_I32, OP_SORT_F64, OP_SORT_KV_I32, OP_PARTITION_I32, OP_SORT_SEGMENTED_I32, OP_SORT_U32, OP_SORT_I64,
 OP_SORT_KV_F64, OP_SORT_SEGMENTED_F64) = range(9)
PIVOT_AUTO, PIVOT_MEDIAN3, PIVOT_NINTHER, PIVOT_SAMPLE = range(4)

_STATUS = {0: "HS_OK", -1: "HS_EINVAL", -2: "HS_ENOMEM", -3: "HS_EHIP", -4: "HS_EWORKSPACE",
           -5: "HS_EUNSUPPORTED", -6: "HS_EINTERNAL"}


class HSortError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


METHOD_PLAIN, METHOD_LEARNED = 0, 1
DRIVER_AUTO, DRIVER_HOST, DRIVER_PERSISTENT = 0, 1, 2
LEARN_FORCE_MODEL, LEARN_FORCE_SAMPLE = 1, 2


class Stats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int64), ("bytes_alg", ctypes.c_int64),
                ("keys_partitioned", ctypes.c_int64), ("tasks", ctypes.c_int64),
                ("max_depth", ctypes.c_int64), ("fallback_used", ctypes.c_int32),
                ("splitters", ctypes.c_int32), ("bucket_imbalance", ctypes.c_double),
                ("partition_ms", ctypes.c_double), ("local_ms", ctypes.c_double),
                ("partition_launches", ctypes.c_int64),
                ("model_imbalance", ctypes.c_double), ("sample_imbalance", ctypes.c_double),
                ("learn_ms", ctypes.c_double), ("multiway_ms", ctypes.c_double),
                ("final_loss", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Opts(ctypes.Structure):
    _fields_ = [("pivot_rule", ctypes.c_int32), ("local_T", ctypes.c_int32),
                ("method", ctypes.c_int32), ("learn_flags", ctypes.c_int32),
                ("train_steps", ctypes.c_int32), ("sample_log2", ctypes.c_int32),
                ("learning_rate", ctypes.c_float), ("driver", ctypes.c_int32),
                ("spin_limit", ctypes.c_int32), ("leaf", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("inplace", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64

_SIGS = {
    "hs_sort_i32": ([_P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_sort_f64": ([_P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_sort_kv_i32": ([_P, _P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_sort_kv_f64": ([_P, _P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_sort_u32": ([_P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_sort_i64": ([_P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_argsort_i32": ([_P, _P, _P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_argsort_f64": ([_P, _P, _P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_partition_i32": ([_P, _I64, ctypes.c_int32, _P, _P, _P], ctypes.c_int),
    "hs_sort_i32_noalloc": ([_P, _I64, _P], ctypes.c_int),
    "hs_sort_segmented_i32": ([_P, _I64, _P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_sort_segmented_f64": ([_P, _I64, _P, _I64, _P, _P, _P], ctypes.c_int),
    "hs_workspace_size": ([ctypes.c_int, _I64, _I64, _P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hs_mlp_forward_f32": ([_P, _P, _I64, _P, _P], ctypes.c_int),
    "hs_mlp_grad_f32": ([_P, _P, _P, _I64, _P, _P], ctypes.c_int),
    "hs_mlp_train_f32": ([_P, _P, _I64, ctypes.c_int32, ctypes.c_float, ctypes.c_uint64, _P, _P, _P],
                         ctypes.c_int),
    "hs_multiway_partition_f64": ([_P, _I64, _P, ctypes.c_int32, _P, _P], ctypes.c_int),
    "hs_learn_debug_f64": ([_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "hs_plan_create": ([ctypes.c_int, _I64, _I64, _P, _P], ctypes.c_int),
    "hs_plan_exec": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "hs_plan_check": ([_P, _P], ctypes.c_int),
    "hs_plan_destroy": ([_P], None),
    "hs_autotune": ([ctypes.c_int, _P, _P, _I64, _P, _I64, _P, _P, _P, _P], ctypes.c_int),
    "hs_last_error": ([], ctypes.c_char_p),
    "hs_version": ([], ctypes.c_int),
}


def lib() -> ctypes.CDLL:
    """Load libhsort.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1704_08579_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int):
    if rc != HS_OK:
        msg = lib().hs_last_error()
        raise HSortError(rc, msg.decode() if msg else "")


def _torch():
    import torch
    return torch


def _stream_handle(t) -> int:
    torch = _torch()
    return torch.cuda.current_stream(t.device).cuda_stream


def _require(t, dtypes, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dim() != 1:
        raise ValueError(f"{name} must be one-dimensional")


def _opts_ptr(opts):
    return None if opts is None else ctypes.addressof(opts)


def _sort_fn(dtype):
    torch = _torch()
    return {torch.int32: "hs_sort_i32", torch.float64: "hs_sort_f64", torch.uint32: "hs_sort_u32",
            torch.int64: "hs_sort_i64"}[dtype]


def sort_(t, opts: Opts | None = None, stats: bool = False):
    """Sort a 1-D int32, uint32, int64 or float64 CUDA tensor in place
    (float64 by IEEE totalOrder)."""
    torch = _torch()
    _require(t, (torch.int32, torch.float64, torch.uint32, torch.int64), "t")
    st = Stats() if stats else None
    with torch.cuda.device(t.device):
        fn = getattr(lib(), _sort_fn(t.dtype))
        _check(fn(t.data_ptr(), t.numel(), _opts_ptr(opts), None if st is None else ctypes.addressof(st),
                  _stream_handle(t)))
    return st.as_dict() if st is not None else t


def argsort(keys, opts: Opts | None = None, stats: bool = False, out=None):
    """Stable argsort of a 1-D int32 or float64 (totalOrder) CUDA tensor:
    returns (sorted keys, int32 indices) with keys[idx] == sorted keys and
    equal keys in input order.  `keys` is left as it is unless
    out=(keys, idx) names it."""
    torch = _torch()
    _require(keys, (torch.int32, torch.float64), "keys")
    if out is None:
        ko = torch.empty_like(keys)
        idx = torch.empty(keys.shape, dtype=torch.int32, device=keys.device)
    else:
        ko, idx = out
        _require(ko, (keys.dtype,), "out[0]")
        _require(idx, (torch.int32,), "out[1]")
        if ko.numel() != keys.numel() or idx.numel() != keys.numel():
            raise ValueError("out tensors must have the size of keys")
    fn = lib().hs_argsort_i32 if keys.dtype == torch.int32 else lib().hs_argsort_f64
    st = Stats() if stats else None
    with torch.cuda.device(keys.device):
        _check(fn(keys.data_ptr(), ko.data_ptr(), idx.data_ptr(), keys.numel(), _opts_ptr(opts),
                  None if st is None else ctypes.addressof(st), _stream_handle(keys)))
    return (ko, idx, st.as_dict()) if st is not None else (ko, idx)


def sort_kv_(keys, vals, opts: Opts | None = None, stats: bool = False):
    """Sort (key, value) pairs held in two tensors, in place, by key: int32 or
    float64 keys (totalOrder), int32 values; equal keys end up ordered by
    their values' bits as unsigned integers."""
    torch = _torch()
    _require(keys, (torch.int32, torch.float64), "keys")
    _require(vals, (torch.int32,), "vals")
    if keys.numel() != vals.numel() or keys.device != vals.device:
        raise ValueError("keys and vals must have the same size and device")
    fn = lib().hs_sort_kv_i32 if keys.dtype == torch.int32 else lib().hs_sort_kv_f64
    st = Stats() if stats else None
    with torch.cuda.device(keys.device):
        _check(fn(keys.data_ptr(), vals.data_ptr(), keys.numel(), _opts_ptr(opts),
                  None if st is None else ctypes.addressof(st), _stream_handle(keys)))
    return st.as_dict() if st is not None else (keys, vals)


def partition_(t, pivot: int, count_out=None, opts: Opts | None = None):
    """Partition an int32 tensor in place: t[:k] <= pivot < t[k:].  The count
    k is written on the device into `count_out` (a 1-element int64 tensor,
    allocated if None), which is returned; no host synchronisation."""
    torch = _torch()
    _require(t, (torch.int32,), "t")
    if count_out is None:
        count_out = torch.empty(1, dtype=torch.int64, device=t.device)
    _require(count_out, (torch.int64,), "count_out")
    with torch.cuda.device(t.device):
        _check(lib().hs_partition_i32(t.data_ptr(), t.numel(), int(pivot), count_out.data_ptr(),
                                      _opts_ptr(opts), _stream_handle(t)))
    return count_out


def sort_segmented_(t, offsets, opts: Opts | None = None, stats: bool = False):
    """Sort every segment t[off[i]:off[i+1]] of an int32 or float64 tensor in
    place.  `offsets` is an int64 CUDA tensor of nseg+1 entries, off[0] = 0,
    non-decreasing, off[-1] = t.numel()."""
    torch = _torch()
    _require(t, (torch.int32, torch.float64), "t")
    _require(offsets, (torch.int64,), "offsets")
    fn = lib().hs_sort_segmented_i32 if t.dtype == torch.int32 else lib().hs_sort_segmented_f64
    st = Stats() if stats else None
    with torch.cuda.device(t.device):
        _check(fn(t.data_ptr(), t.numel(), offsets.data_ptr(), offsets.numel() - 1, _opts_ptr(opts),
                  None if st is None else ctypes.addressof(st), _stream_handle(t)))
    return st.as_dict() if st is not None else t


def workspace_size(op: int, n: int, nseg: int = 0, opts: Opts | None = None) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().hs_workspace_size(op, n, nseg, _opts_ptr(opts), ctypes.byref(out)))
    return int(out.value)


# ---------------------------------------------------------------- learned splitters

MLP_NPARAM = 1153


def learned_opts(steps: int = 0, sample_log2: int = 0, lr: float = 0.0, seed: int = 0, flags: int = 0) -> Opts:
    """Options selecting the learned-splitter method."""
    o = Opts()
    o.method = METHOD_LEARNED
    o.train_steps = steps
    o.sample_log2 = sample_log2
    o.learning_rate = lr
    o.seed = seed
    o.learn_flags = flags
    return o


def mlp_forward(params, z):
    """F(z) for a float32 CUDA tensor z with the 1153 float32 parameters."""
    torch = _torch()
    _require(params, (torch.float32,), "params")
    _require(z, (torch.float32,), "z")
    out = torch.empty_like(z)
    with torch.cuda.device(z.device):
        _check(lib().hs_mlp_forward_f32(params.data_ptr(), z.data_ptr(), z.numel(), out.data_ptr(),
                                        _stream_handle(z)))
    return out


def mlp_grad(params, z, y):
    """Gradient of the mean squared error over (z, y) (1153 float32 values)."""
    torch = _torch()
    for t, nm in ((params, "params"), (z, "z"), (y, "y")):
        _require(t, (torch.float32,), nm)
    g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=z.device)
    with torch.cuda.device(z.device):
        _check(lib().hs_mlp_grad_f32(params.data_ptr(), z.data_ptr(), y.data_ptr(), z.numel(), g.data_ptr(),
                                     _stream_handle(z)))
    return g


def mlp_train(z, y, steps: int, lr: float, seed: int):
    """Train from the seeded initialisation; returns (params, per-step losses)."""
    torch = _torch()
    _require(z, (torch.float32,), "z")
    _require(y, (torch.float32,), "y")
    p = torch.empty(MLP_NPARAM, dtype=torch.float32, device=z.device)
    loss = torch.empty(max(1, steps), dtype=torch.float32, device=z.device)
    with torch.cuda.device(z.device):
        _check(lib().hs_mlp_train_f32(z.data_ptr(), y.data_ptr(), z.numel(), steps, lr, seed, p.data_ptr(),
                                      loss.data_ptr(), _stream_handle(z)))
    return p, loss[:steps]


def multiway_partition_(keys, splitters):
    """Split a float64 tensor in place by distinct increasing splitters (a
    uint64-valued int64 tensor of totalOrder keys); returns the bucket starts
    (int32 tensor of 2k+2 entries, read as uint32)."""
    torch = _torch()
    _require(keys, (torch.float64,), "keys")
    _require(splitters, (torch.int64,), "splitters")
    k = splitters.numel()
    starts = torch.empty(2 * k + 2, dtype=torch.int32, device=keys.device)
    with torch.cuda.device(keys.device):
        _check(lib().hs_multiway_partition_f64(keys.data_ptr(), keys.numel(), splitters.data_ptr(), k,
                                               starts.data_ptr(), _stream_handle(keys)))
    return starts


class LearnReport(ctypes.Structure):
    _fields_ = [("scale", ctypes.c_double), ("mu", ctypes.c_double), ("sd", ctypes.c_double),
                ("smin", ctypes.c_uint64),
                ("smax", ctypes.c_uint64), ("m", ctypes.c_int32), ("h", ctypes.c_int32), ("k", ctypes.c_int32),
                ("use_model", ctypes.c_int32), ("model_imbalance", ctypes.c_float),
                ("sample_imbalance", ctypes.c_float), ("final_loss", ctypes.c_float), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


NB_MAX = 511  # buckets of 255 distinct splitters, equality buckets included


def learn_debug(keys, opts: Opts | None = None):
    """The learned front end of a float64 sort on its own (hs_learn_debug_f64;
    `keys` is not changed).  Returns a dict: the report's fields, and CUDA
    tensors params (1153 float32), model_split, sample_split, chosen (255
    totalOrder words as int64; the first k of chosen are used), holdout (2^14
    words), train_sorted (the sorted training sample, float64) and counts
    (2 x 511 int32: held-out bucket counts, model then order statistics)."""
    torch = _torch()
    _require(keys, (torch.float64,), "keys")
    dev = keys.device
    m = 1 << (opts.sample_log2 if opts is not None and opts.sample_log2 > 0 else 16)
    out = {"params": torch.empty(MLP_NPARAM, dtype=torch.float32, device=dev),
           "model_split": torch.empty(255, dtype=torch.int64, device=dev),
           "sample_split": torch.empty(255, dtype=torch.int64, device=dev),
           "chosen": torch.empty(255, dtype=torch.int64, device=dev),
           "holdout": torch.empty(1 << 14, dtype=torch.int64, device=dev),
           "train_sorted": torch.empty(m, dtype=torch.float64, device=dev),
           "counts": torch.zeros(2 * NB_MAX, dtype=torch.int32, device=dev)}
    rep = LearnReport()
    with torch.cuda.device(dev):
        _check(lib().hs_learn_debug_f64(keys.data_ptr(), keys.numel(), _opts_ptr(opts), out["params"].data_ptr(),
                                        out["model_split"].data_ptr(), out["sample_split"].data_ptr(),
                                        out["chosen"].data_ptr(), out["holdout"].data_ptr(),
                                        out["train_sorted"].data_ptr(), out["counts"].data_ptr(),
                                        ctypes.addressof(rep), _stream_handle(keys)))
    out.update(rep.as_dict())
    return out


# ---------------------------------------------------------------- plans and the autotuner

class TuneReport(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("outputs_equal", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("local_T", ctypes.c_int32), ("leaf", ctypes.c_int32), ("pivot_rule", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


def _sort_args(keys, vals=None, offsets=None):
    """(op, keys ptr, vals ptr, n, offsets ptr, nseg) of a sort over tensors."""
    torch = _torch()
    if offsets is not None:
        _require(keys, (torch.int32, torch.float64), "keys")
        _require(offsets, (torch.int64,), "offsets")
        op = OP_SORT_SEGMENTED_I32 if keys.dtype == torch.int32 else OP_SORT_SEGMENTED_F64
        return op, keys.data_ptr(), None, keys.numel(), offsets.data_ptr(), offsets.numel() - 1
    if vals is not None:
        _require(keys, (torch.int32, torch.float64), "keys")
        _require(vals, (torch.int32,), "vals")
        if keys.numel() != vals.numel() or keys.device != vals.device:
            raise ValueError("keys and vals must have the same size and device")
        op = OP_SORT_KV_I32 if keys.dtype == torch.int32 else OP_SORT_KV_F64
        return op, keys.data_ptr(), vals.data_ptr(), keys.numel(), None, 0
    _require(keys, (torch.int32, torch.float64, torch.uint32, torch.int64), "keys")
    op = {torch.int32: OP_SORT_I32, torch.float64: OP_SORT_F64, torch.uint32: OP_SORT_U32,
          torch.int64: OP_SORT_I64}[keys.dtype]
    return op, keys.data_ptr(), None, keys.numel(), None, 0


class Plan:
    """A sort of a fixed shape captured into a HIP graph (hs_plan_*).

    Built from example tensors (their dtype and sizes fix the shape; they are
    also the default buffers of ``run``).  ``run()`` sorts the default
    tensors, ``run(keys, vals=..., offsets=...)`` other tensors of the same
    shape, on the current stream."""

    def __init__(self, keys, vals=None, offsets=None, opts: Opts | None = None):
        torch = _torch()
        op, _, _, n, _, nseg = _sort_args(keys, vals, offsets)
        self._op, self._n, self._nseg = op, n, nseg
        self._default = (keys, vals, offsets)
        self._bound = None
        self._plan = ctypes.c_void_p()
        self.device = keys.device
        with torch.cuda.device(keys.device):
            _check(lib().hs_plan_create(op, n, nseg, _opts_ptr(opts), ctypes.byref(self._plan)))

    def run(self, keys=None, vals=None, offsets=None):
        torch = _torch()
        if keys is None:
            keys, vals, offsets = self._default
        op, kp, vp, n, op_off, nseg = _sort_args(keys, vals, offsets)
        if (op, n, nseg) != (self._op, self._n, self._nseg):
            raise ValueError("tensors of another shape than the plan's")
        if keys.device != self.device:
            raise ValueError("tensors on another device than the plan's")
        self._bound = (keys, vals, offsets)  # kept alive while a replay may use them
        with torch.cuda.device(self.device):
            _check(lib().hs_plan_exec(self._plan, kp, vp, op_off, torch.cuda.current_stream(self.device).cuda_stream))
        return self

    def check(self):
        torch = _torch()
        with torch.cuda.device(self.device):
            _check(lib().hs_plan_check(self._plan, torch.cuda.current_stream(self.device).cuda_stream))

    def close(self):
        if getattr(self, "_plan", None) and self._plan.value:
            lib().hs_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(keys, vals=None, offsets=None, opts: Opts | None = None):
    """Tune the knobs for this sort (the tensors are left unchanged); returns
    (tuned Opts, report dict)."""
    torch = _torch()
    op, kp, vp, n, op_off, nseg = _sort_args(keys, vals, offsets)
    best = Opts()
    rep = TuneReport()
    with torch.cuda.device(keys.device):
        _check(lib().hs_autotune(op, kp, vp, n, op_off, nseg, _opts_ptr(opts), ctypes.byref(best), ctypes.byref(rep),
                                 _stream_handle(keys)))
    return best, rep.as_dict()
