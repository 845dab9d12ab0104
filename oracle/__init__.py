"""CPU oracle for the hybrid quicksort + bitonic sort (TEST INFRASTRUCTURE).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path (the HIP
library and its Python binding) never imports, links or calls it.

The arithmetic lives in ``hsort_oracle.c`` (plain scalar C, one thread); this
module only loads the shared object built from it and marshals numpy arrays.
Every function cites the part of the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "hsort_oracle.c"), os.path.join(_HERE, "learned_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_CTX_SRC = os.path.join(_HERE, "std_sort_context.cpp")
_CTX_LIB = os.path.join(_HERE, "libstdsort_context.so")

_I64 = ctypes.c_int64
_P = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O2, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(map(os.path.getmtime, _SRCS)):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    if force or not os.path.exists(_CTX_LIB) or os.path.getmtime(_CTX_LIB) < os.path.getmtime(_CTX_SRC):
        tmp = _CTX_LIB + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _CTX_SRC])
        os.replace(tmp, _CTX_LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(map(os.path.getmtime, _SRCS)):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        for name, args, res in [
            ("oracle_sort_i32", [_P, _I64, _I64], _I64),
            ("oracle_sort_f64", [_P, _I64, _I64], _I64),
            ("oracle_sort_kv_i32", [_P, _P, _I64, _I64], _I64),
            ("oracle_sort_kv_f64", [_P, _P, _I64, _I64], _I64),
            ("oracle_argsort_f64", [_P, _P, _I64, _I64], _I64),
            ("oracle_sort_u32", [_P, _I64, _I64], _I64),
            ("oracle_sort_i64", [_P, _I64, _I64], _I64),
            ("oracle_argsort_i32", [_P, _P, _I64, _I64], _I64),
            ("oracle_sort_segmented_i32", [_P, _P, _I64, _I64], _I64),
            ("oracle_sort_segmented_f64", [_P, _P, _I64, _I64], _I64),
            ("oracle_partition_le_i32", [_P, _I64, ctypes.c_int32], _I64),
            ("oracle_bitonic_apply", [_P, _P, ctypes.c_int], None),
            ("oracle_bitonic_exhaustive_failures", [ctypes.c_int], _I64),
            ("oracle_bitonic_merger_failures", [ctypes.c_int], _I64),
            ("oracle_key_f64", [ctypes.c_uint64], ctypes.c_uint64),
            ("oracle_unkey_f64", [ctypes.c_uint64], ctypes.c_uint64),
            ("oracle_splitmix64_at", [ctypes.c_uint64, ctypes.c_uint64], ctypes.c_uint64),
            ("oracle_sample_indices", [ctypes.c_uint64, _I64, _I64, _P], None),
            ("oracle_mlp_nparam", [], _I64),
            ("oracle_mlp_init", [ctypes.c_uint64, _P], None),
            ("oracle_mlp_forward", [_P, _P, _I64, _P], None),
            ("oracle_mlp_loss_grad", [_P, _P, _P, _I64, _P], ctypes.c_double),
            ("oracle_adam_step", [_P, _P, _P, _P, _I64, ctypes.c_double], None),
            ("oracle_feature_scale", [_P, _I64], ctypes.c_double),
            ("oracle_feature_stats", [_P, _I64, ctypes.c_double, _P, _P], None),
            ("oracle_training_points", [_I64, _P], _I64),
            ("oracle_mlp_train", [ctypes.c_uint64, _P, _P, _I64, _I64, ctypes.c_double, _P, _P], None),
            ("oracle_invert_one_f64", [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _P, _I64,
                                       ctypes.c_double], _I64),
            ("oracle_invert_f64", [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _P, _I64, ctypes.c_int,
                                   _P], None),
            ("oracle_dedupe", [_P, _I64, _P], _I64),
            ("oracle_bucket_hist", [_P, _I64, _P, _I64, _P], None),
            ("oracle_keys_f64", [_P, _I64, _P], None),
        ]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


LEAF = 256  # the paper's sort bound: 16 vectors of 16 int32


def sort_i32(keys: np.ndarray, leaf: int = LEAF) -> np.ndarray:
    a = np.ascontiguousarray(keys, dtype=np.int32).copy()
    if lib().oracle_sort_i32(_ptr(a), a.size, leaf) < 0:
        raise MemoryError("oracle_sort_i32")
    return a


def sort_i32_depth(keys: np.ndarray, leaf: int = LEAF):
    a = np.ascontiguousarray(keys, dtype=np.int32).copy()
    d = lib().oracle_sort_i32(_ptr(a), a.size, leaf)
    return a, d


def sort_f64(keys: np.ndarray, leaf: int = LEAF) -> np.ndarray:
    """Sort float64 values by IEEE totalOrder; returns the permuted values."""
    a = np.ascontiguousarray(keys, dtype=np.float64).copy().view(np.uint64)
    if lib().oracle_sort_f64(_ptr(a), a.size, leaf) < 0:
        raise MemoryError("oracle_sort_f64")
    return a.view(np.float64)


def sort_u32(keys: np.ndarray, leaf: int = LEAF) -> np.ndarray:
    a = np.ascontiguousarray(keys, dtype=np.uint32).copy()
    if lib().oracle_sort_u32(_ptr(a), a.size, leaf) < 0:
        raise MemoryError("oracle_sort_u32")
    return a


def sort_i64(keys: np.ndarray, leaf: int = LEAF) -> np.ndarray:
    a = np.ascontiguousarray(keys, dtype=np.int64).copy()
    if lib().oracle_sort_i64(_ptr(a), a.size, leaf) < 0:
        raise MemoryError("oracle_sort_i64")
    return a


def argsort_i32(keys: np.ndarray, leaf: int = LEAF):
    """Stable argsort: (sorted keys, int32 positions of them in `keys`)."""
    k = np.ascontiguousarray(keys, dtype=np.int32).copy()
    idx = np.empty(k.size, dtype=np.int32)
    if lib().oracle_argsort_i32(_ptr(k), _ptr(idx), k.size, leaf) < 0:
        raise MemoryError("oracle_argsort_i32")
    return k, idx


def sort_kv_i32(keys: np.ndarray, vals: np.ndarray, leaf: int = LEAF):
    k = np.ascontiguousarray(keys, dtype=np.int32).copy()
    v = np.ascontiguousarray(vals, dtype=np.int32).copy()
    assert k.size == v.size
    if lib().oracle_sort_kv_i32(_ptr(k), _ptr(v), k.size, leaf) < 0:
        raise MemoryError("oracle_sort_kv_i32")
    return k, v


def sort_kv_f64(keys: np.ndarray, vals: np.ndarray, leaf: int = LEAF):
    """(float64 key, int32 value) pairs by the key's totalOrder; returns the
    permuted keys and values."""
    k = np.ascontiguousarray(keys, dtype=np.float64).copy().view(np.uint64)
    v = np.ascontiguousarray(vals, dtype=np.int32).copy()
    assert k.size == v.size
    if lib().oracle_sort_kv_f64(_ptr(k), _ptr(v), k.size, leaf) < 0:
        raise MemoryError("oracle_sort_kv_f64")
    return k.view(np.float64), v


def argsort_f64(keys: np.ndarray, leaf: int = LEAF):
    """Stable argsort by totalOrder: (sorted keys, int32 positions of them in `keys`)."""
    k = np.ascontiguousarray(keys, dtype=np.float64).copy().view(np.uint64)
    idx = np.empty(k.size, dtype=np.int32)
    if lib().oracle_argsort_f64(_ptr(k), _ptr(idx), k.size, leaf) < 0:
        raise MemoryError("oracle_argsort_f64")
    return k.view(np.float64), idx


def sort_segmented_i32(keys: np.ndarray, offsets: np.ndarray, leaf: int = LEAF) -> np.ndarray:
    k = np.ascontiguousarray(keys, dtype=np.int32).copy()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    if lib().oracle_sort_segmented_i32(_ptr(k), _ptr(off), off.size - 1, leaf) < 0:
        raise MemoryError("oracle_sort_segmented_i32")
    return k


def sort_segmented_f64(keys: np.ndarray, offsets: np.ndarray, leaf: int = LEAF) -> np.ndarray:
    """Every [off[i], off[i+1]) of a float64 array sorted on its own (totalOrder)."""
    a = np.ascontiguousarray(keys, dtype=np.float64).copy().view(np.uint64)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    if lib().oracle_sort_segmented_f64(_ptr(a), _ptr(off), off.size - 1, leaf) < 0:
        raise MemoryError("oracle_sort_segmented_f64")
    return a.view(np.float64)


def partition_le_i32(keys: np.ndarray, pivot: int):
    a = np.ascontiguousarray(keys, dtype=np.int32).copy()
    k = lib().oracle_partition_le_i32(_ptr(a), a.size, int(pivot))
    return a, int(k)


def bitonic_apply(keys: np.ndarray, vals: np.ndarray | None = None):
    k = np.ascontiguousarray(keys, dtype=np.uint64).copy()
    logn = int(k.size).bit_length() - 1
    assert (1 << logn) == k.size
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.int32).copy()
    lib().oracle_bitonic_apply(_ptr(k), None if v is None else _ptr(v), logn)
    return k if v is None else (k, v)


def bitonic_exhaustive_failures(logn: int) -> int:
    return int(lib().oracle_bitonic_exhaustive_failures(logn))


def bitonic_merger_failures(logn: int) -> int:
    return int(lib().oracle_bitonic_merger_failures(logn))


def key_f64(bits: int) -> int:
    return int(lib().oracle_key_f64(bits))


def unkey_f64(key: int) -> int:
    return int(lib().oracle_unkey_f64(key))


# ---------------------------------------------------------------- learned splitters

NPARAM = 1153


def splitmix64_at(seed: int, k: int) -> int:
    return int(lib().oracle_splitmix64_at(seed & (2 ** 64 - 1), k))


def sample_indices(seed: int, n: int, m: int) -> np.ndarray:
    idx = np.empty(m, dtype=np.int64)
    lib().oracle_sample_indices(seed & (2 ** 64 - 1), n, m, _ptr(idx))
    return idx


def mlp_init(seed: int) -> np.ndarray:
    p = np.empty(NPARAM, dtype=np.float64)
    lib().oracle_mlp_init(seed & (2 ** 64 - 1), _ptr(p))
    return p


def mlp_forward(p, z) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty(z.size, dtype=np.float64)
    lib().oracle_mlp_forward(_ptr(p), _ptr(z), z.size, _ptr(out))
    return out


def mlp_loss_grad(p, z, y):
    p = np.ascontiguousarray(p, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = np.empty(NPARAM, dtype=np.float64)
    loss = lib().oracle_mlp_loss_grad(_ptr(p), _ptr(z), _ptr(y), z.size, _ptr(g))
    return float(loss), g


def adam_step(p, mom, vel, grad, t: int, lr: float):
    """In-place Adam update of float64 arrays p, mom, vel."""
    for a in (p, mom, vel):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    g = np.ascontiguousarray(grad, dtype=np.float64)
    lib().oracle_adam_step(_ptr(p), _ptr(mom), _ptr(vel), _ptr(g), int(t), float(lr))


def feature_scale(sorted_x) -> float:
    """Scale s of the model's feature asinh(x / s), from the sorted sample."""
    x = np.ascontiguousarray(sorted_x, dtype=np.float64)
    return float(lib().oracle_feature_scale(_ptr(x), x.size))


def feature_stats(x, s: float = 1.0):
    """Mean and population standard deviation of asinh(x / s)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    mu = ctypes.c_double()
    sd = ctypes.c_double()
    lib().oracle_feature_stats(_ptr(x), x.size, float(s), ctypes.addressof(mu), ctypes.addressof(sd))
    return mu.value, sd.value


def training_points(m: int) -> np.ndarray:
    """Ranks of the training set in a sorted sample of m keys."""
    r = np.empty(min(m, 4096), dtype=np.int64)
    nt = lib().oracle_training_points(m, _ptr(r))
    return r[:nt]


def mlp_train(seed: int, z, y, steps: int, lr: float):
    z = np.ascontiguousarray(z, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    p = np.empty(NPARAM, dtype=np.float64)
    losses = np.empty(steps, dtype=np.float64)
    lib().oracle_mlp_train(seed & (2 ** 64 - 1), _ptr(z), _ptr(y), z.size, steps, lr, _ptr(p), _ptr(losses))
    return p, losses


def invert_f64(p, s: float, mu: float, sd: float, sorted_keys, nb: int = 256) -> np.ndarray:
    """Splitters: for j = 1..nb-1 the smallest key of the sorted sample (order
    words) with F >= j/nb, then the running maximum."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    sk = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    out = np.empty(nb - 1, dtype=np.uint64)
    lib().oracle_invert_f64(_ptr(p), s, mu, sd, _ptr(sk), sk.size, nb, _ptr(out))
    return out


def invert_one_f64(p, s: float, mu: float, sd: float, sorted_keys, q: float) -> int:
    """Rank of one splitter before the running maximum (the bisection's
    crossing of q over the sorted sample)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    sk = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    return int(lib().oracle_invert_one_f64(_ptr(p), s, mu, sd, _ptr(sk), sk.size, q))


def dedupe(s) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.uint64)
    d = np.empty(max(1, s.size), dtype=np.uint64)
    k = lib().oracle_dedupe(_ptr(s), s.size, _ptr(d))
    return d[:k].copy()


def bucket_hist(keys, d) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    d = np.ascontiguousarray(d, dtype=np.uint64)
    counts = np.empty(2 * d.size + 1, dtype=np.int64)
    lib().oracle_bucket_hist(_ptr(keys), keys.size, _ptr(d) if d.size else None, d.size, _ptr(counts))
    return counts


def f64_order_keys(x) -> np.ndarray:
    """Order words (IEEE totalOrder keys) of float64 values."""
    bits = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)
    out = np.empty(bits.size, dtype=np.uint64)
    lib().oracle_keys_f64(_ptr(bits), bits.size, _ptr(out))
    return out


_ctx = None


def std_sort_context(a: np.ndarray) -> np.ndarray:
    """GNU std::sort of an int32 or float64 array on the calling thread (the
    paper's comparison library, timed by the benchmark for context only)."""
    global _ctx
    if _ctx is None:
        if not os.path.exists(_CTX_LIB):
            build(force=False)
        _ctx = ctypes.CDLL(_CTX_LIB)
        for nm in ("context_std_sort_i32", "context_std_sort_f64"):
            getattr(_ctx, nm).argtypes = [_P, _I64]
            getattr(_ctx, nm).restype = None
    out = np.ascontiguousarray(a).copy()
    fn = _ctx.context_std_sort_i32 if out.dtype == np.int32 else _ctx.context_std_sort_f64
    if out.dtype not in (np.int32, np.float64):
        raise TypeError(out.dtype)
    fn(_ptr(out), out.size)
    return out
