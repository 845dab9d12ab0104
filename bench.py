#!/usr/bin/env python3
"""Benchmark of the gfx950 hybrid quicksort + bitonic sort.

One step sorts one batch of synthetic keys resident in HBM.  The default
workload sorts four arrays of 2^27 float64 keys (uniform [0,1), N(0,1),
already sorted, reverse sorted; IEEE totalOrder), so one step is 2^29 keys.

Printed: ONE JSON line with the sort throughput (Gkeys/s, from HIP events on
the sort stream around each sort call; the restore copy of the unsorted input
before each sort is outside the events), the roofline of the dominant kernel
(the partition pass: algorithmic bytes 2*s per key per level over its event
time), and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME] [--extra]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

CONFIGS = {
    # name: (kind, n, distributions or None, seed, description)
    "f64_2e27": ("f64", 1 << 27, ["uniform", "normal", "sorted", "reverse"], 2,
                 "sort_f64, 2^27 float64 keys x 4 distributions (uniform [0,1), N(0,1), sorted, reverse)"),
    "i32_2e20": ("i32", 1 << 20, None, 1, "sort_i32, 2^20 int32 keys uniform over the full range"),
    "i32_2e28": ("i32", 1 << 28, None, 1, "sort_i32, 2^28 int32 keys uniform over the full range"),
    "kv_2e28": ("kv", 1 << 28, None, 4,
                "sort_kv_i32, 2^28 int32 pairs, 2^16 distinct keys, values = original index"),
    "kvf64_2e27": ("kvf64", 1 << 27, None, 6,
                   "sort_kv_f64, 2^27 (float64 key, int32 value) pairs, 2^16 distinct N(0,1) keys, "
                   "values = original index"),
    "seg_A": ("seg", 200000, (16, 1 << 13), 5,
              "sort_segmented_i32, 200,000 int32 arrays, sizes log-uniform in [16, 2^13]"),
    "seg_B": ("seg", 2840, (16, 1 << 20), 5,
              "sort_segmented_i32, 2,840 int32 arrays, sizes log-uniform in [16, 2^20]"),
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

# configurations sorted with the partition levels in place
INPLACE = {"f64_2e27_inplace", "i32_2e28_inplace"}

# configurations sorted with the learned-splitter method: name -> learn_flags
LEARNED = {"learned_2e28": 0, "sampled_2e28_learned_inputs": 2}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(name):
    import numpy as np

    import workloads
    kind, n, extra, seed, _ = CONFIGS[name]
    if kind == "f64":
        return [("f64", workloads.f64(n, d, seed=seed)) for d in extra]
    if kind == "i32":
        return [("i32", workloads.uniform_i32(n, seed=seed))]
    if kind == "kv":
        k, v = workloads.kv_dup_i32(n, seed=seed)
        return [("kv", (k, v))]
    if kind == "kvf64":
        k, v = workloads.kv_dup_f64(n, seed=seed)
        return [("kvf64", (k, v))]
    if kind == "seg":
        lo, hi = extra
        off = workloads.segment_offsets(n, lo, hi, seed=seed)
        return [("seg", (workloads.uniform_i32(int(off[-1]), seed=seed + 1), off.astype(np.int64)))]
    raise ValueError(kind)


class Case:
    """One array of the step: pristine device copy + work buffers."""

    def __init__(self, kind, data, torch):
        self.kind = kind
        dev = "cuda"
        if kind in ("f64", "i32"):
            self.src = torch.from_numpy(data).to(dev)
            self.work = torch.empty_like(self.src)
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
            self.work = torch.empty_like(self.src)
            self.off = torch.from_numpy(off).to(dev)
            self.n = k.size
            self.s = 4

    def restore(self):
        self.work.copy_(self.src)
        if self.kind in ("kv", "kvf64"):
            self.vwork.copy_(self.vsrc)

    def sort(self, hs, opts=None):
        if getattr(self, "plan", None) is not None:
            return self.plan.run()
        if self.kind in ("f64", "i32"):
            return hs.sort_(self.work, opts=opts, stats=True)
        if self.kind in ("kv", "kvf64"):
            return hs.sort_kv_(self.work, self.vwork, opts=opts, stats=True)
        return hs.sort_segmented_(self.work, self.off, opts=opts, stats=True)


def run_gpu(name, steps, warmup, driver=0):
    import torch

    import paper_1704_08579_amd as hs
    hs.lib()
    inputs = make_inputs(name)
    dists = CONFIGS[name][2] if CONFIGS[name][0] == "f64" else [None] * len(inputs)
    cases = [Case(k, d, torch) for k, d in inputs]
    del inputs
    opts = hs.learned_opts(seed=100, flags=LEARNED[name]) if name in LEARNED else hs.Opts()
    opts.driver = driver
    opts.inplace = 1 if name in INPLACE else 0
    learn = {d: [] for d in dists} if name in LEARNED else None
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
        # stats of one eager sort with the tuned knobs (the graph cannot read them back)
        c.restore()
        seg_stats = c.sort(hs, tuned)
        c.plan = hs.Plan(c.work, offsets=c.off, opts=tuned)
        graph = dict(tune_report=report, tune_s=round(tune_s, 2),
                     knobs=dict(local_T=tuned.local_T, leaf=tuned.leaf, pivot_rule=tuned.pivot_rule))
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    sort_ms = []
    acc = dict(bytes_alg=0, keys_part=0, part_ms=0.0, part_launches=0, local_ms=0.0, local_keys=0)
    for step in range(warmup + steps):
        timed = step >= warmup
        if step == warmup:
            torch.cuda.synchronize()
            t_wall = time.perf_counter()
        ms_step = 0.0
        for c, dist in zip(cases, dists):
            c.restore()
            ev0.record()
            st = c.sort(hs, opts)
            ev1.record()
            ev1.synchronize()
            ms_step += ev0.elapsed_time(ev1)
            if graph is not None:
                c.plan.check()
                st = seg_stats
            if timed and learn is not None:
                learn[dist].append(dict(ms=ev0.elapsed_time(ev1), learn_ms=st["learn_ms"],
                                        multiway_ms=st["multiway_ms"], fallback_used=st["fallback_used"],
                                        splitters=st["splitters"], model_imbalance=st["model_imbalance"],
                                        sample_imbalance=st["sample_imbalance"], final_loss=st["final_loss"],
                                        bytes_per_key=st["bytes_alg"] / c.n))
            if timed:
                acc["bytes_alg"] += st["bytes_alg"]
                acc["keys_part"] += st["keys_partitioned"]
                acc["part_ms"] += st["partition_ms"]
                acc["part_launches"] += st["partition_launches"]
                acc["local_ms"] += st["local_ms"]
                acc["local_keys"] += c.n
        if timed:
            sort_ms.append(ms_step)
        log(f"[bench] {name} step {step} ({'timed' if timed else 'warmup'}): {ms_step:.3f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    keys_step = sum(c.n for c in cases)
    s = cases[0].s
    ms = sum(sort_ms) / len(sort_ms)
    part_bytes = 2 * s * acc["keys_part"]
    part_gbs = part_bytes / (acc["part_ms"] * 1e-3) / 1e9 if acc["part_ms"] > 0 else 0.0
    local_gbs = 2 * s * acc["local_keys"] / (acc["local_ms"] * 1e-3) / 1e9 if acc["local_ms"] > 0 else 0.0
    total_s = sum(sort_ms) * 1e-3
    return dict(
        name=name, keys_per_step=keys_step, ms_per_step=ms, wall_ms_per_step=wall * 1e3 / steps,
        gkeys=keys_step / (ms * 1e-3) / 1e9,
        bytes_per_key=acc["bytes_alg"] / (keys_step * steps),
        whole_sort_roofline=acc["bytes_alg"] / total_s / 1e9 / HBM_PEAK_GBS,
        partition=dict(gbs=part_gbs, ms_per_step=acc["part_ms"] / steps,
                       launches_per_step=acc["part_launches"] / steps,
                       bytes_per_launch=part_bytes / max(1, acc["part_launches"]),
                       avg_launch_ms=acc["part_ms"] / max(1, acc["part_launches"])),
        local=dict(gbs=local_gbs, ms_per_step=acc["local_ms"] / steps),
        elem_bytes=s,
        learned=None if learn is None else {
            d: {k: round(sum(r[k] for r in v) / len(v), 4) for k in v[0]} for d, v in learn.items()},
        graph=graph,
    )


def measured_traffic(name, kernel):
    """HBM traffic per launch of the dominant kernel from the committed
    rocprofv3 --pmc summary for this workload, or None when there is none or
    the kernel source has changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_{name}.md")
    src = os.path.join(ROOT, "paper_1704_08579_amd", "csrc", "hs_kernels.hpp")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    sha = re.search(r"^source_sha256: ([0-9a-f]+)", txt, re.M)
    val = re.search(r"^traffic_bytes_per_launch: ([0-9]+)", txt, re.M)
    if not sha or not val:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != sha.group(1):
        return None
    return int(val.group(1))


def cpu_baseline(name):
    """The oracle (single thread, as written) on a bounded sample of the
    workload: the first 2^27 keys of the first array of the step (about
    15 s for float64 on one host core)."""
    import numpy as np

    import oracle
    kind, n, extra, seed, _ = CONFIGS[name]
    inputs = make_inputs(name)
    kind0, data = inputs[0]
    m = min(n, 1 << 27)
    t0 = time.perf_counter()
    if kind0 == "f64":
        oracle.sort_f64(data[:m])
        what = f"first 2^{m.bit_length() - 1} keys of the {extra[0]} float64 array"
    elif kind0 == "i32":
        oracle.sort_i32(data[:m])
        what = f"first 2^{m.bit_length() - 1} keys of the int32 array"
    elif kind0 == "kv":
        oracle.sort_kv_i32(data[0][:m], data[1][:m])
        what = f"first 2^{m.bit_length() - 1} pairs"
    elif kind0 == "kvf64":
        oracle.sort_kv_f64(data[0][:m], data[1][:m])
        what = f"first 2^{m.bit_length() - 1} float64 key/value pairs"
    else:
        k, off = data
        nseg = int(np.searchsorted(off, m, side="right")) - 1
        sub = off[: nseg + 1]
        oracle.sort_segmented_i32(k[: int(sub[-1])], sub)
        m = int(sub[-1])
        what = f"first {nseg} segments ({m} keys)"
    dt = time.perf_counter() - t0
    return {"value": m / dt / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": what + f", {dt:.1f} s on one host core ({platform.processor() or platform.machine()}, "
                             f"os.cpu_count()={os.cpu_count()})"}


def run_small(reps=40):
    """Small arrays: latency of one sort per size (GPU time between events on
    the sort stream, and host time from the call to the sort's completion),
    and batched sorts of many equal-size arrays in one segmented call."""
    import statistics

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
    ap.add_argument("--config", default="f64_2e27", choices=sorted(CONFIGS))
    ap.add_argument("--extra", action="store_true", help="also run the int32, key/value and batched configs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small", action="store_true",
                    help="also measure small arrays: per-size latency and batched throughput")
    ap.add_argument("--driver", choices=["persistent", "host"], default="host",
                    help="partition levels in one persistent launch, or one launch per level")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU; --gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)

    driver = 2 if args.driver == "persistent" else 1
    r = run_gpu(args.config, args.steps, args.warmup, driver)
    extra = {}
    if args.extra:
        for nm in ["i32_2e28", "kv_2e28", "kvf64_2e27", "seg_A", "seg_B", "i32_2e20", "learned_2e28",
                   "sampled_2e28_learned_inputs", "plain_2e28_learned_inputs", "f64_2e27_inplace",
                   "i32_2e28_inplace"]:
            if nm == args.config:
                continue
            e = run_gpu(nm, max(3, args.steps // 2), 1, driver)
            extra[nm] = {"gkeys_per_s": round(e["gkeys"], 3), "ms_per_step": round(e["ms_per_step"], 3),
                         "bytes_per_key": round(e["bytes_per_key"], 1),
                         "partition_gbs": round(e["partition"]["gbs"], 1),
                         "whole_sort_roofline_frac": round(e["whole_sort_roofline"], 4),
                         "workload": CONFIGS[nm][4]}
            if e["learned"]:
                extra[nm]["per_distribution"] = e["learned"]
            if e["graph"]:
                extra[nm]["graph"] = e["graph"]
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.config)

    kind, n, _, _, desc = CONFIGS[args.config]
    p = r["partition"]
    out = {
        "metric": "sorted Gkeys/s + HBM roofline %",
        "value": round(r["gkeys"], 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "u64", "i32": "u32", "kv": "u64", "kvf64": "u128", "seg": "u32"}[kind],
        "data": "synthetic",
        "config": {"workload": desc, "keys_per_step": r["keys_per_step"],
                   "bytes_per_key": round(r["bytes_per_key"], 1),
                   "whole_sort_roofline_frac": round(r["whole_sort_roofline"], 4),
                   "wall_ms_per_step_incl_restore": round(r["wall_ms_per_step"], 3),
                   "local_sort_gbs": round(r["local"]["gbs"], 1),
                   "local_sort_ms_per_step": round(r["local"]["ms_per_step"], 3),
                   "partition_ms_per_step": round(p["ms_per_step"], 3),
                   "partition_launches_per_step": p["launches_per_step"]},
        "roofline": {"bound": "hbm",
                     "kernel": ("k_levels (every partition level of a sort in one persistent launch)" if driver == 2
                                else "k_partition (one partition level per launch)"),
                     "achieved": round(p["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(p["gbs"] / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.config, "k_levels" if driver == 2 else "k_partition"),
                     "bytes_per_launch": round(p["bytes_per_launch"]),
                     "avg_launch_ms": round(p["avg_launch_ms"], 4)},
        "cpu_baseline": cpu,
    }
    if r["learned"]:
        out["config"]["learned_per_distribution"] = r["learned"]
    if extra:
        out["extra"] = extra
    if args.small:
        out["small_arrays"] = run_small()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
