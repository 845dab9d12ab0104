#!/usr/bin/env python3
"""Benchmark of the gfx950 hybrid quicksort + bitonic sort.

One step sorts one array of 2^28 int32 keys (uniform over the full range)
resident in HBM; `value` is its median throughput over the timed steps.
Beside it, with the same protocol, the same run measures the other 2^28
sorts (float64 keys by totalOrder, int32 key/value pairs with 2^16 distinct
keys), the learned-splitter form next to the plain one on a lognormal(0,2)
float64 input, the batched form (200,000 int32 arrays, one graph replay),
the 2^20 int32 case and the four 2^27 float64 distributions.

Protocol per workload: W untimed warm-up sorts, then K timed sorts, each
preceded by a device copy that restores the unsorted input (outside the
events); the time of a sort is the HIP-event time around the call on the
sort stream; median, min and max are reported.  Statistics (levels, keys
partitioned, per-launch event times of the partition pass) come from extra
instrumented sorts after the timed ones.  Every output is checked against
numpy (outside the timed region), and the outputs of all timed sorts of a
workload must be identical.  The CPU oracle (one pinned host core) and GNU
std::sort are timed on a bounded sample of the headline input.

Printed: ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME] [--extra] [--small]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

CONFIGS = {
    # name: (kind, n, distributions or segment bounds, seed, description)
    "i32_2e28": ("i32", 1 << 28, None, 1, "sort_i32, 2^28 int32 keys uniform over the full range"),
    "f64_2e28": ("f64", 1 << 28, ["uniform"], 2, "sort_f64, 2^28 float64 keys uniform on [0,1) (totalOrder)"),
    "kv_2e28": ("kv", 1 << 28, None, 4,
                "sort_kv_i32, 2^28 int32 pairs, 2^16 distinct keys, values = original index"),
    "f64_2e27": ("f64", 1 << 27, ["uniform", "normal", "sorted", "reverse"], 2,
                 "sort_f64, 2^27 float64 keys x 4 distributions (uniform [0,1), N(0,1), sorted, reverse)"),
    "i32_2e20": ("i32", 1 << 20, None, 1, "sort_i32, 2^20 int32 keys uniform over the full range"),
    "i32_2e20_plan": ("i32", 1 << 20, None, 1,
                      "sort_i32, 2^20 int32 keys uniform over the full range, one graph replay (hs_plan_exec)"),
    "kvf64_2e27": ("kvf64", 1 << 27, None, 6,
                   "sort_kv_f64, 2^27 (float64 key, int32 value) pairs, 2^16 distinct N(0,1) keys, "
                   "values = original index"),
    "seg_A": ("seg", 200000, (16, 1 << 13), 5,
              "sort_segmented_i32, 200,000 int32 arrays, sizes log-uniform in [16, 2^13], one autotuned graph replay"),
    "seg_B": ("seg", 2840, (16, 1 << 20), 5,
              "sort_segmented_i32, 2,840 int32 arrays, sizes log-uniform in [16, 2^20], one autotuned graph replay"),
    "learned_2e28_lognormal": ("f64", 1 << 28, ["lognormal"], 6,
                               "sort_f64 with learned splitters (training included), 2^28 lognormal(0,2) float64 keys"),
    "plain_2e28_lognormal": ("f64", 1 << 28, ["lognormal"], 6,
                             "sort_f64 (plain method) on the input of learned_2e28_lognormal"),
    "learned_2e28": ("f64", 1 << 28, ["lognormal", "zipf", "mixture"], 6,
                     "sort_f64 with learned splitters (training included), 2^28 float64 keys x 3 distributions "
                     "(lognormal(0,2), Zipf s=1.1 over 2^24, 8-Gaussian mixture)"),
    "sampled_2e28_learned_inputs": ("f64", 1 << 28, ["lognormal", "zipf", "mixture"], 6,
                                    "sort_f64 with the multiway pass driven by the sample's order statistics "
                                    "(no training) on the inputs of learned_2e28"),
    "plain_2e28_learned_inputs": ("f64", 1 << 28, ["lognormal", "zipf", "mixture"], 6,
                                  "sort_f64 (plain method) on the inputs of learned_2e28"),
    "f64_2e27_inplace": ("f64", 1 << 27, ["uniform", "normal", "sorted", "reverse"], 2,
                         "sort_f64 with the partition levels in place (no second copy of the keys), "
                         "2^27 float64 keys x 4 distributions"),
    "i32_2e28_inplace": ("i32", 1 << 28, None, 1,
                         "sort_i32 with the partition levels in place, 2^28 int32 keys uniform over the full range"),
}

HEADLINE = "i32_2e28"
# measured beside the headline in a default run
BESIDE = ["f64_2e28", "kv_2e28", "plain_2e28_lognormal", "learned_2e28_lognormal", "seg_A", "i32_2e20",
          "i32_2e20_plan", "f64_2e27"]
# measured too with --extra
EXTRA = ["kvf64_2e27", "seg_B", "learned_2e28", "sampled_2e28_learned_inputs", "plain_2e28_learned_inputs",
         "f64_2e27_inplace", "i32_2e28_inplace"]

# configurations sorted by replaying a graph plan of a single array
PLANNED = {"i32_2e20_plan"}
# configurations sorted with the partition levels in place
INPLACE = {"f64_2e27_inplace", "i32_2e28_inplace"}
# configurations sorted with the learned-splitter method: name -> learn_flags
LEARNED = {"learned_2e28": 0, "learned_2e28_lognormal": 0, "sampled_2e28_learned_inputs": 2}

DTYPE = {"f64": "u64", "i32": "u32", "kv": "u64", "kvf64": "u128", "seg": "u32"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(name):
    import numpy as np

    import workloads
    kind, n, extra, seed, _ = CONFIGS[name]
    if kind == "f64":
        return [("f64", d, workloads.f64(n, d, seed=seed)) for d in extra]
    if kind == "i32":
        return [("i32", None, workloads.uniform_i32(n, seed=seed))]
    if kind == "kv":
        return [("kv", None, workloads.kv_dup_i32(n, seed=seed))]
    if kind == "kvf64":
        return [("kvf64", None, workloads.kv_dup_f64(n, seed=seed))]
    if kind == "seg":
        lo, hi = extra
        off = workloads.segment_offsets(n, lo, hi, seed=seed)
        return [("seg", None, (workloads.uniform_i32(int(off[-1]), seed=seed + 1), off.astype(np.int64)))]
    raise ValueError(kind)


# ---------------------------------------------------------------- output checks (numpy, outside the timing)

def _f64_sorted_bits(x):
    """float64 values sorted by IEEE totalOrder, as uint64 bits."""
    import numpy as np
    u = x.view(np.uint64)
    k = np.where(u >> np.uint64(63), ~u, u | np.uint64(1 << 63))
    k.sort()
    return np.where(k >> np.uint64(63), k & np.uint64((1 << 63) - 1), ~k)


def check_output(kind, host_in, out):
    """Raise if `out` (numpy) is not the sorted form of `host_in`."""
    import numpy as np
    if kind == "i32":
        if not np.array_equal(out, np.sort(host_in)):
            raise AssertionError("int32 output differs from numpy's sort")
    elif kind == "f64":
        if not np.array_equal(out.view(np.uint64), _f64_sorted_bits(host_in)):
            raise AssertionError("float64 output differs from the totalOrder sort")
    elif kind in ("kv", "kvf64"):
        k_in, _ = host_in
        k_out, v_out = out
        ref = np.sort(k_in) if kind == "kv" else _f64_sorted_bits(k_in).view(np.float64)
        if not np.array_equal(k_out.view(np.uint8), ref.view(np.uint8)):
            raise AssertionError("key/value keys differ from numpy's sort")
        idx = v_out.astype(np.int64)
        if idx.min() < 0 or idx.max() >= k_in.size or np.bincount(idx, minlength=k_in.size).max() != 1:
            raise AssertionError("values are not a permutation of the input positions")
        if not np.array_equal(k_in[idx].view(np.uint8), k_out.view(np.uint8)):
            raise AssertionError("a key lost its value")
    elif kind == "seg":
        k_in, off = host_in
        sid = np.repeat(np.arange(off.size - 1, dtype=np.int64), np.diff(off))
        comb = (sid << 32) | (k_in.astype(np.int64) + (1 << 31))
        comb.sort()
        ref = ((comb & 0xFFFFFFFF) - (1 << 31)).astype(np.int32)
        if not np.array_equal(out, ref):
            raise AssertionError("segmented output differs from per-segment sorts")
    else:
        raise ValueError(kind)


# ---------------------------------------------------------------- one workload

class Case:
    """One array of a workload: pristine device copy and work buffers."""

    def __init__(self, kind, dist, data, torch):
        self.kind, self.dist, self.host = kind, dist, data
        dev = "cuda"
        self.off = None
        if kind in ("f64", "i32"):
            self.src = torch.from_numpy(data).to(dev)
            self.work = torch.empty_like(self.src)
            self.vsrc = None
            self.n = data.size
            self.s = data.itemsize
        elif kind in ("kv", "kvf64"):
            k, v = data
            self.src = torch.from_numpy(k).to(dev)
            self.vsrc = torch.from_numpy(v).to(dev)
            self.work = torch.empty_like(self.src)
            self.vwork = torch.empty_like(self.vsrc)
            self.n = k.size
            self.s = 8 if kind == "kv" else 16  # bytes of the order word a pair travels as
        else:
            k, off = data
            self.src = torch.from_numpy(k).to(dev)
            self.vsrc = None
            self.work = torch.empty_like(self.src)
            self.off = torch.from_numpy(off).to(dev)
            self.n = k.size
            self.s = 4
        self.plan = None
        self.first = None  # output of the first timed sort (device copy)

    def restore(self):
        self.work.copy_(self.src)
        if self.vsrc is not None:
            self.vwork.copy_(self.vsrc)

    def sort(self, hs, opts, stats):
        if self.plan is not None:
            self.plan.run()
            return None
        if self.kind in ("f64", "i32"):
            return hs.sort_(self.work, opts=opts, stats=stats)
        if self.kind in ("kv", "kvf64"):
            return hs.sort_kv_(self.work, self.vwork, opts=opts, stats=stats)
        return hs.sort_segmented_(self.work, self.off, opts=opts, stats=stats)

    def output(self):
        if self.vsrc is not None:
            return (self.work.cpu().numpy(), self.vwork.cpu().numpy())
        return self.work.cpu().numpy()

    def keep_first(self):
        self.first = [self.work.clone()] + ([self.vwork.clone()] if self.vsrc is not None else [])

    def same_as_first(self, torch):
        cur = [self.work] + ([self.vwork] if self.vsrc is not None else [])
        return all(torch.equal(a, b) for a, b in zip(self.first, cur))


def run_workload(name, steps, warmup, driver=0, stat_runs=3):
    """Time one workload; returns a dict of its measurements."""
    import torch

    import paper_1704_08579_amd as hs
    hs.lib()
    t_in = time.perf_counter()
    cases = [Case(k, d, data, torch) for k, d, data in make_inputs(name)]
    log(f"[bench] {name}: inputs ready ({time.perf_counter() - t_in:.1f} s)")
    opts = hs.learned_opts(seed=100, flags=LEARNED[name]) if name in LEARNED else hs.Opts()
    opts.driver = driver
    opts.inplace = 1 if name in INPLACE else 0
    graph = None
    if CONFIGS[name][0] == "seg":
        # batched segmented sort: autotuned knobs, one graph replay per sort
        c = cases[0]
        c.restore()
        base = hs.Opts()
        base.driver = hs.DRIVER_PERSISTENT
        t0 = time.perf_counter()
        tuned, report = hs.autotune(c.work, offsets=c.off, opts=base)
        tune_s = time.perf_counter() - t0
        c.plan = hs.Plan(c.work, offsets=c.off, opts=tuned)
        graph = dict(tune_report=report, tune_s=round(tune_s, 2),
                     knobs=dict(local_T=tuned.local_T, leaf=tuned.leaf, pivot_rule=tuned.pivot_rule))
        stat_opts = tuned
    elif name in PLANNED:
        c = cases[0]
        c.restore()
        c.plan = hs.Plan(c.work)
        graph = dict(plan="hs_plan_create / hs_plan_exec, default knobs")
        stat_opts = opts
    else:
        stat_opts = opts
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # the copy ceiling: the device copy that restores the first array's input
    # (reads and writes its bytes once), best of five
    copy_ms = []
    for _ in range(5):
        ev0.record()
        cases[0].restore()
        ev1.record()
        ev1.synchronize()
        copy_ms.append(ev0.elapsed_time(ev1))
    c0 = cases[0]
    copy_bytes = 2 * (c0.src.numel() * c0.src.element_size() +
                      (c0.vsrc.numel() * c0.vsrc.element_size() if c0.vsrc is not None else 0))
    copy_gbs = copy_bytes / (min(copy_ms) * 1e-3) / 1e9
    step_ms = []
    case_ms = [[] for _ in cases]
    torch.cuda.synchronize()
    for step in range(warmup + steps):
        timed = step >= warmup
        ms_step = 0.0
        for ci, c in enumerate(cases):
            c.restore()
            ev0.record()
            c.sort(hs, opts, False)
            ev1.record()
            ev1.synchronize()
            ms_step += ev0.elapsed_time(ev1)
            if timed:
                case_ms[ci].append(ev0.elapsed_time(ev1))
            if c.plan is not None:
                c.plan.check()
            if step == warmup:
                c.keep_first()
        if timed:
            step_ms.append(ms_step)
        log(f"[bench] {name} step {step} ({'timed' if timed else 'warmup'}): {ms_step:.3f} ms")
    # every timed sort gave the same output; the last one is checked against numpy
    t_chk = time.perf_counter()
    for c in cases:
        if not c.same_as_first(torch):
            raise AssertionError(f"{name}: timed sorts gave different outputs")
        check_output(c.kind, c.host, c.output())
        c.first = None
    log(f"[bench] {name}: outputs checked against numpy ({time.perf_counter() - t_chk:.1f} s)")
    # instrumented sorts (per-level events inside the library), outside the timing
    acc = dict(bytes_alg=0, keys_part=0, part_ms=0.0, part_launches=0, local_ms=0.0, local_keys=0, levels=0)
    learn = {}
    for _ in range(stat_runs):
        for c in cases:
            c.restore()
            if c.plan is not None:
                saved, c.plan = c.plan, None
                st = c.sort(hs, stat_opts, True)
                c.plan = saved
            else:
                st = c.sort(hs, opts, True)
            acc["bytes_alg"] += st["bytes_alg"]
            acc["keys_part"] += st["keys_partitioned"]
            acc["part_ms"] += st["partition_ms"]
            acc["part_launches"] += st["partition_launches"]
            acc["local_ms"] += st["local_ms"]
            acc["local_keys"] += c.n
            acc["levels"] += st["passes"]
            if name in LEARNED:
                learn.setdefault(c.dist, []).append(dict(
                    learn_ms=st["learn_ms"], multiway_ms=st["multiway_ms"], fallback_used=st["fallback_used"],
                    splitters=st["splitters"], model_imbalance=st["model_imbalance"],
                    sample_imbalance=st["sample_imbalance"], final_loss=st["final_loss"],
                    bytes_per_key=st["bytes_alg"] / c.n,
                    gkeys_without_front_end=c.n / ((statistics.median(case_ms[cases.index(c)]) - st["learn_ms"])
                                                   * 1e-3) / 1e9))
    if graph is not None and CONFIGS[name][0] == "seg":
        # the plain comparison of a batched sort: one hs_sort_i32 call per array,
        # over the first 2000 arrays
        c = cases[0]
        c.restore()
        off = c.host[1]
        ks = 0
        torch.cuda.synchronize()
        ev0.record()
        for i in range(min(2000, len(off) - 1)):
            a, b = int(off[i]), int(off[i + 1])
            if b - a >= 2:
                hs.sort_(c.work[a:b])
            ks += b - a
        ev1.record()
        ev1.synchronize()
        graph["eager_loop"] = dict(arrays=min(2000, len(off) - 1), keys=ks,
                                   gkeys_per_s=round(ks / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 3),
                                   what="one hs_sort_i32 call per array, the first arrays of the batch")
    keys_step = sum(c.n for c in cases)
    s = cases[0].s
    med = statistics.median(step_ms)
    nst = stat_runs
    part_bytes = 2 * s * acc["keys_part"]
    part_gbs = part_bytes / (acc["part_ms"] * 1e-3) / 1e9 if acc["part_ms"] > 0 else 0.0
    bytes_per_step = acc["bytes_alg"] / nst
    out = dict(
        name=name, kind=cases[0].kind, keys_per_step=keys_step, elem_bytes=s,
        median_ms=med, min_ms=min(step_ms), max_ms=max(step_ms), runs=len(step_ms),
        gkeys=keys_step / (med * 1e-3) / 1e9,
        bytes_per_key=bytes_per_step / keys_step,
        whole_sort_roofline=bytes_per_step / (med * 1e-3) / 1e9 / HBM_PEAK_GBS,
        levels_per_sort=acc["levels"] / (nst * len(cases)),
        partition=dict(gbs=part_gbs, ms_per_step=acc["part_ms"] / nst,
                       launches_per_step=acc["part_launches"] / nst,
                       bytes_per_launch=part_bytes / max(1, acc["part_launches"]),
                       avg_launch_ms=acc["part_ms"] / max(1, acc["part_launches"])),
        local=dict(ms_per_step=acc["local_ms"] / nst,
                   gbs=2 * s * acc["local_keys"] / (acc["local_ms"] * 1e-3) / 1e9 if acc["local_ms"] > 0 else 0.0),
        graph=graph,
        learned={d: {k: round(sum(r[k] for r in v) / len(v), 4) for k in v[0]} for d, v in learn.items()} or None,
        copy_gbs=copy_gbs,
        ideal_bytes_per_key=ideal_bytes_per_key(name, s),
    )
    for c in cases:
        if c.plan is not None:
            c.plan.close()
    del cases
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def ideal_bytes_per_key(name, s):
    """Bytes per key of a plain sort with perfect splits: 2 s per level,
    ceil(log2(n / T)) levels, plus the on-chip sort (T: the on-chip limit),
    for a single array sorted by the plain method; None otherwise."""
    kind, n = CONFIGS[name][0], CONFIGS[name][1]
    if kind == "seg" or name in LEARNED:
        return None
    T = 4096 if kind == "kvf64" else 8192
    levels = max(0, math.ceil(math.log2(n / T)))
    return 2 * s * (levels + 1)


def summary(r):
    """The fields of one workload printed beside the headline."""
    d = {"workload": CONFIGS[r["name"]][4], "gkeys_per_s": round(r["gkeys"], 3),
         "ms_per_step": {"median": round(r["median_ms"], 4), "min": round(r["min_ms"], 4),
                         "max": round(r["max_ms"], 4), "runs": r["runs"]},
         "keys_per_step": r["keys_per_step"], "bytes_per_key": round(r["bytes_per_key"], 1),
         "whole_sort_roofline_frac": round(r["whole_sort_roofline"], 4),
         "partition_gbs": round(r["partition"]["gbs"], 1),
         "partition_ms_per_step": round(r["partition"]["ms_per_step"], 3),
         "local_sort_ms_per_step": round(r["local"]["ms_per_step"], 3),
         "levels_per_sort": round(r["levels_per_sort"], 2), "output_checked": True,
         "copy_ceiling_gbs": round(r["copy_gbs"], 1)}
    if r["ideal_bytes_per_key"]:
        d["ideal_bytes_per_key"] = r["ideal_bytes_per_key"]
    if CONFIGS[r["name"]][1] * r["elem_bytes"] <= (8 << 20):
        d["note"] = "the input fits the on-chip caches (L2 and MALL): the roofline fractions are not HBM figures"
    if r["learned"]:
        d["per_distribution"] = r["learned"]
    if r["graph"]:
        d["graph"] = r["graph"]
    return d


def partition_source_sha():
    """sha256 of the source the partition pass is built from: the device
    primitives, and the shared types, tile geometry and partition-pass
    sections of the kernel header."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1704_08579_amd", "csrc")
    dev = open(os.path.join(csrc, "hs_device.hpp")).read()
    k = open(os.path.join(csrc, "hs_kernels.hpp")).read()
    mark = "// ---------------------------------------------------------------- "
    head = k[:k.index(mark + "grid barrier")]
    part = k[k.index(mark + "partition pass"):k.index(mark + "finalize")]
    return hashlib.sha256((dev + head + part).encode()).hexdigest()


def measured_traffic(name, kernel):
    """HBM traffic per launch of the dominant kernel from the committed
    rocprofv3 --pmc summary for this workload, or None when there is none or
    the kernel's source has changed since the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_{name}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    sha = re.search(r"^partition_source_sha256: ([0-9a-f]+)", txt, re.M)
    val = re.search(r"^traffic_bytes_per_launch: ([0-9]+)", txt, re.M)
    if not sha or not val or sha.group(1) != partition_source_sha():
        return None
    return int(val.group(1))


def cpu_baseline(name, log2_sample=26):
    """The oracle (single thread, as written) on the first 2^26 keys of the
    workload's first array, on one pinned host core (about 15 s for int32),
    and GNU std::sort once on the same sample for context."""
    import numpy as np

    import oracle
    kind, n, extra, seed, _ = CONFIGS[name]
    _, dist, data = make_inputs(name)[0]
    m = min(n, 1 << log2_sample)
    prev = os.sched_getaffinity(0)
    core = min(prev)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        if kind == "f64":
            sample = data[:m]
            out = oracle.sort_f64(sample)
            what = f"first 2^{m.bit_length() - 1} keys of the {dist} float64 array"
        elif kind == "i32":
            sample = data[:m]
            out = oracle.sort_i32(sample)
            what = f"first 2^{m.bit_length() - 1} keys of the int32 array"
        elif kind == "kv":
            sample = data[0][:m]
            out, _ = oracle.sort_kv_i32(sample, data[1][:m])
            what = f"first 2^{m.bit_length() - 1} pairs"
        else:
            raise ValueError(f"no CPU baseline for {name}")
        dt = time.perf_counter() - t0
        t1 = time.perf_counter()
        ref = oracle.std_sort_context(sample)
        dt_std = time.perf_counter() - t1
    finally:
        os.sched_setaffinity(0, prev)
    if not np.array_equal(out.view(np.uint8), ref.view(np.uint8)) and kind != "f64":
        raise AssertionError("the oracle and std::sort disagree on the CPU sample")
    host = f"{platform.processor() or platform.machine()}, os.cpu_count()={os.cpu_count()}"
    return {"value": m / dt / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": what + f", {dt:.1f} s on one pinned host core ({host})",
            "std_sort_context": {"value": m / dt_std / 1e9, "unit": "Gkeys/s", "cores": 1,
                                 "seconds": round(dt_std, 2),
                                 "note": "GNU std::sort on the same sample and core (the paper's comparison "
                                         "library; context only)"}}


def run_small(reps=40):
    """Small arrays: latency of one sort per size (GPU time between events on
    the sort stream, and host time from the call to the sort's completion),
    and batched sorts of many equal-size arrays in one segmented call."""
    import torch

    import paper_1704_08579_amd as hs
    import workloads
    hs.lib()
    dev = torch.device("cuda")
    out = {"single": {}, "batched_i32": {}}
    sizes = [2, 16, 64, 256, 512, 1024, 2048, 8192, 65536]
    for kind in ("i32", "f64", "kv", "kvf64"):
        rows = {}
        for n in sizes:
            if kind in ("f64", "kvf64"):
                src = torch.from_numpy(workloads.f64(n, "uniform", seed=n)).to(dev)
            else:
                src = torch.from_numpy(workloads.uniform_i32(n, seed=n)).to(dev)
            t = src.clone()
            v = torch.arange(n, dtype=torch.int32, device=dev) if kind in ("kv", "kvf64") else None
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            gpu_us, wall_us = [], []
            for r in range(reps + 5):
                t.copy_(src)
                torch.cuda.synchronize()
                w0 = time.perf_counter()
                e0.record()
                if v is not None:
                    hs.sort_kv_(t, v)
                else:
                    hs.sort_(t)
                e1.record()
                e1.synchronize()
                w1 = time.perf_counter()
                if r >= 5:
                    gpu_us.append(e0.elapsed_time(e1) * 1e3)
                    wall_us.append((w1 - w0) * 1e6)
            rows[str(n)] = {"gpu_us": round(statistics.median(gpu_us), 1),
                            "call_to_done_us": round(statistics.median(wall_us), 1)}
        out["single"][kind] = rows
    total = 1 << 22
    for s in (16, 64, 256, 1024, 4096):
        nseg = total // s
        off = torch.arange(0, (nseg + 1) * s, s, dtype=torch.int64, device=dev)
        src = torch.from_numpy(workloads.uniform_i32(nseg * s, seed=s)).to(dev)
        t = src.clone()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for r in range(8):
            t.copy_(src)
            e0.record()
            hs.sort_segmented_(t, off)
            e1.record()
            e1.synchronize()
            if r >= 2:
                ms.append(e0.elapsed_time(e1))
        m = statistics.median(ms)
        out["batched_i32"][str(s)] = {"arrays": nseg, "ms": round(m, 3), "gkeys_per_s": round(nseg * s / m / 1e6, 2)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default=HEADLINE, choices=sorted(CONFIGS),
                    help="the workload of `value` (default: int32 2^28)")
    ap.add_argument("--only", action="store_true", help="measure --config alone, nothing beside it")
    ap.add_argument("--extra", action="store_true", help="also measure the remaining workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small", action="store_true",
                    help="also measure small arrays: per-size latency and batched throughput")
    ap.add_argument("--driver", choices=["auto", "persistent", "host"], default="auto",
                    help="partition levels in one persistent launch, or one launch per level")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the sort runs on one GPU; --gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        print("bench.py: --steps must be at least 1", file=sys.stderr)
        sys.exit(2)

    driver = {"auto": 0, "host": 1, "persistent": 2}[args.driver]
    r = run_workload(args.config, args.steps, args.warmup, driver)
    beside = {}
    names = [] if args.only else [nm for nm in BESIDE + (EXTRA if args.extra else []) if nm != args.config]
    for nm in names:
        beside[nm] = summary(run_workload(nm, args.steps, min(args.warmup, 2), driver))
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.config)

    p = r["partition"]
    persistent = driver == 2
    kernel = "k_levels" if persistent else "k_partition"
    out = {
        "metric": "sorted Gkeys/s at 2^28 + HBM roofline %",
        "value": round(r["gkeys"], 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["median_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[r["kind"]],
        "data": "synthetic",
        "config": {"workload": CONFIGS[args.config][4], "keys_per_step": r["keys_per_step"],
                   "timing": {"statistic": "median", "min_ms": round(r["min_ms"], 4),
                              "max_ms": round(r["max_ms"], 4), "runs": r["runs"]},
                   "bytes_per_key": round(r["bytes_per_key"], 1),
                   "whole_sort_roofline_frac": round(r["whole_sort_roofline"], 4),
                   "levels_per_sort": round(r["levels_per_sort"], 2),
                   "local_sort_gbs": round(r["local"]["gbs"], 1),
                   "local_sort_ms_per_step": round(r["local"]["ms_per_step"], 3),
                   "partition_ms_per_step": round(p["ms_per_step"], 3),
                   "partition_launches_per_step": p["launches_per_step"],
                   "ideal_bytes_per_key": r["ideal_bytes_per_key"],
                   "output_checked": True},
        "roofline": {"bound": "hbm",
                     "kernel": ("k_levels (every partition level of a sort in one persistent launch)" if persistent
                                else "k_partition (one partition level per launch)"),
                     "achieved": round(p["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(p["gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.config, kernel),
                     "bytes_per_launch": round(p["bytes_per_launch"]),
                     "avg_launch_ms": round(p["avg_launch_ms"], 4),
                     "whole_sort_frac": round(r["whole_sort_roofline"], 4),
                     "copy_ceiling_gbs": round(r["copy_gbs"], 1),
                     "frac_of_copy_ceiling": round(p["gbs"] / r["copy_gbs"], 4)},
        "cpu_baseline": cpu,
    }
    if r["learned"]:
        out["config"]["learned_per_distribution"] = r["learned"]
    if r["graph"]:
        out["config"]["graph"] = r["graph"]
    if beside:
        out["beside"] = beside
    if args.small:
        out["small_arrays"] = run_small()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
