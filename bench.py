#!/usr/bin/env python3
"""Throughput of the MI355X sample sort on the paper's workload shape.

One step = one complete sort (every level and the base case) of one batch of
synthetic keys already resident in HBM.  The default workload is n = 2^28
uniform uint64 keys with two sample-sort levels of k = 256 groups and
overpartitioning b = 4.  Prints ONE JSON line with the throughput, the
roofline of the dominant kernel (timed live with HIP events on the sort's
stream) and the oracle timed on the host.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1410_6754_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

# name -> (n, key type, distribution, with payload, sort parameters, config index)
WORKLOADS = {
    "uniform_u64_2^28": (1 << 28, W.KEY_U64, "uniform", False,
                         dict(levels=2, k=256, overpartition_b=4), 2),
    "sorted_u64_2^28": (1 << 28, W.KEY_U64, "sorted", False,
                        dict(levels=2, k=256, overpartition_b=4), 2),
    "reversed_u64_2^28": (1 << 28, W.KEY_U64, "reversed", False,
                          dict(levels=2, k=256, overpartition_b=4), 2),
    "uniform_u64_2^20": (1 << 20, W.KEY_U64, "uniform", False,
                         dict(levels=1, k=256, overpartition_b=1, samples_per_bucket=16,
                              base_cutoff=1024), 1),
    "pairs_few_2^27": (1 << 27, W.KEY_U64, "few", True, dict(), 3),
    "pairs_zipf_2^27": (1 << 27, W.KEY_U64, "zipf", True, dict(), 3),
    "pairs_equal_2^27": (1 << 27, W.KEY_U64, "equal", True, dict(), 3),
}
# RLM-sort (recurse-last multiway mergesort) on the same keys: name ->
# (n, key type, distribution, ams_rlm_params fields, config index)
RLM_WORKLOADS = {
    "rlm_uniform_u64_2^28": (1 << 28, W.KEY_U64, "uniform", dict(), 2),
    "rlm_uniform_u64_2^20": (1 << 20, W.KEY_U64, "uniform", dict(), 1),
}
DEFAULT = "uniform_u64_2^28"
# configurations measured by their own routines (one JSON line each)
SPECIAL = {
    "batch_20000": 4,      # 20,000 segments, sizes floor(2^U), U ~ U(8, 20): ~2^31.2 keys
    "batch_2^28": 4,       # the same seeded list truncated at 2^28 keys in total
    "serving": 5,          # Poisson request stream, mixed key types, p50/p99 latency
}


def key_bytes(kt: int) -> int:
    return 8 if kt == W.KEY_U64 else 4


def kernel_source_hash(files=("ams_engine.hip", "ams_device.h")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1410_6754_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# the sources of RLM-sort's merge kernel
RLM_SOURCES = ("ams_rlm.hip", "ams_device.h")


def measured_traffic(kernel: str, workload: str, files=("ams_engine.hip", "ams_device.h")):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d[workload][kernel]
        if e.get("source_hash") != kernel_source_hash(files):
            return None
        return e["bytes_per_launch"]
    except Exception:
        return None


def host_threads() -> int:
    """Host threads this process may use: its CPU affinity, capped by the
    share OMP_NUM_THREADS names when set."""
    n = len(os.sched_getaffinity(0))
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, n)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(keys: np.ndarray, kt: int, vals, sample_n: int, single_n: int, runs: int = 3):
    """The oracle's mergesort timed on the host: the plain parallel form on
    all host threads over the first sample_n keys (median of `runs` calls:
    the reported value), and the single-threaded form over the first
    single_n keys (one call)."""
    import oracle
    threads = host_threads()
    sample = np.ascontiguousarray(keys[:sample_n])
    times = []
    for _ in range(max(1, runs)):
        t0 = time.perf_counter()
        oracle.oracle_sort_perm_parallel(kt, sample, threads)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    single = np.ascontiguousarray(keys[:single_n])
    sv = None if vals is None else np.ascontiguousarray(vals[:single_n])
    t1 = time.perf_counter()
    oracle.oracle_sort(kt, single, sv)
    dt1 = time.perf_counter() - t1
    return {"value": sample_n / dt / 1e9, "unit": "GKeys/s", "cores": threads, "kind": "oracle",
            "sample": "first %d keys of the workload (2^%d), median of %d calls of the oracle's "
                      "plain parallel mergesort (per-thread chunks, then a pairwise merge tree) "
                      "on %d host threads: %s s" % (sample_n, int(np.log2(sample_n)), len(times),
                                                   threads, ", ".join("%.2f" % t for t in times)),
            "cpu_model": cpu_model(),
            "single_thread": {"value": single_n / dt1 / 1e9, "unit": "GKeys/s", "cores": 1,
                              "sample": "first %d keys (2^%d), the textbook mergesort, %.2f s"
                                        % (single_n, int(np.log2(single_n)), dt1)}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT,
                    choices=sorted(WORKLOADS) + sorted(RLM_WORKLOADS) + sorted(SPECIAL))
    ap.add_argument("--requests", type=int, default=1000, help="serving: requests per load point")
    ap.add_argument("--tune-trials", type=int, default=16,
                    help="batch: parameter sets the autotuner may time")
    ap.add_argument("--no-cpu", action="store_true", help="skip the host oracle timing")
    ap.add_argument("--cpu-sample-log2", type=int, default=27,
                    help="keys the parallel oracle sorts (log2)")
    ap.add_argument("--cpu-single-log2", type=int, default=25,
                    help="keys the single-threaded oracle sorts (log2)")
    ap.add_argument("--cpu-runs", type=int, default=3,
                    help="runs of the parallel oracle (the median is reported)")
    ap.add_argument("--trace-file", default=None, help="write the per-kernel table here")
    ap.add_argument("--params", default=None,
                    help="JSON object of ams_params fields that replace the workload's (sweeps)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device-to-device copy three times (the known-size "
                         "kernel that scales the HBM byte counters), then exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the sort has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.int64, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8,
                          "launches": 3}))
        return 0

    from paper_1410_6754_amd import api

    if args.workload.startswith("batch_"):
        return bench_batch(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload in RLM_WORKLOADS:
        return bench_rlm(args)

    n, kt, dist, pay, pkw, cfg = WORKLOADS[args.workload]
    if args.params:
        pkw = dict(pkw, **json.loads(args.params))
    w = key_bytes(kt) + (4 if pay else 0)
    print("bench: generating %s (n=%d)" % (args.workload, n), file=sys.stderr, flush=True)
    rng = W.rng_for(cfg)
    keys = W.keys(kt, n, rng, dist)
    vals = np.arange(n, dtype=np.uint32) if pay else None

    dev = torch.device("cuda:0")
    d_keys = torch.from_numpy(keys).to(dev)
    d_vals = torch.from_numpy(vals).to(dev) if pay else None
    d_out = torch.empty_like(d_keys)
    d_vout = torch.empty_like(d_vals) if pay else None
    params = api.make_params(**pkw) if pkw else None
    wsb = api.workspace_bytes(kt, n, pay, params)
    ws = api.alloc_workspace(wsb, dev)
    stream = torch.cuda.current_stream()

    def step():
        if pay:
            api.sort_pairs(d_keys, d_vals, d_out, d_vout, params=params, workspace=ws, stream=stream)
        else:
            api.sort_keys(d_keys, d_out, params=params, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("bench: warmup done", file=sys.stderr, flush=True)

    # timed region: K steps between synchronisations; per-kernel events on the
    # sort's stream give the dominant kernel's average launch duration
    api.trace_start()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # an event between consecutive steps as well, for the spread of step times
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev0.record(stream)
    marks[0].record(stream)
    for i in range(args.steps):
        step()
        marks[i + 1].record(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    trace = api.trace_stop()
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    steps_ms = np.array([marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps)])
    step_stats = {"min": round(float(steps_ms.min()), 4),
                  "median": round(float(np.median(steps_ms)), 4),
                  "p90": round(float(np.percentile(steps_ms, 90)), 4)}
    print("bench: timed %d steps, %.3f ms/step (wall %.3f s)" % (args.steps, ms_per_step, wall),
          file=sys.stderr, flush=True)

    # statistics of the sort (every step runs the same plan on the same keys)
    st = api.workspace_stats(ws, stream=stream)
    verified = verify_against_device_sort(kt, d_keys, d_out, d_vout)
    _log("output %s the device reference sort" % ("matches" if verified else "DIFFERS FROM"))

    # per-kernel table (levels folded together)
    per = {}
    for e in trace:
        base = e["name"].split(".")[0]
        d = per.setdefault(base, {"launches": 0, "total_ms": 0.0})
        d["launches"] += e["launches"]
        d["total_ms"] += e["total_ms"]
    kernels = {k: {"launches": v["launches"], "avg_ms": round(v["total_ms"] / v["launches"], 4),
                   "share": round(v["total_ms"] / sum(x["total_ms"] for x in per.values()), 4)}
               for k, v in sorted(per.items(), key=lambda kv: -kv[1]["total_ms"])}
    ceiling = copy_ceiling(api)
    passes, alg = pass_table(trace, st, w, key_bytes(kt), args.steps, ceiling["GB_per_s"])
    # the roofline object: the kernel with the largest time per sort, its
    # algorithmic bytes (keys that took part in its launches) per launch over
    # its average launch duration
    dom = max(per, key=lambda k: per[k]["total_ms"])
    avg_ms = per[dom]["total_ms"] / per[dom]["launches"]
    if dom in alg and alg[dom]["ms"] > 0:
        a = alg[dom]
        achieved = a["bytes"] / (a["ms"] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom, args.workload),
                "algorithmic_bytes_per_launch": int(a["bytes"] / a["launches"]),
                "avg_launch_ms": round(a["ms"] / a["launches"], 4),
                "launches_with_work_per_step": a["launches"] // args.steps}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": None, "traffic": None, "avg_launch_ms": round(avg_ms, 4)}
    levels = [{"level": l, "subproblems": st["subproblems"][l], "keys": st["keys"][l],
               "final_keys": st["final_keys"][l], "max_child": st["max_child"][l],
               "tiles": st["tiles"][l],
               "imbalance_max": round(st["imbalance_max"][l], 4),
               "imbalance_mean": round(st["imbalance_mean"][l], 4)}
              for l in range(st["levels"])]
    leaves = {"leaves": st["leaves"], "big_leaves": st["big_leaves"], "leaf_keys": st["leaf_keys"],
              "copy_keys": st["copy_keys"], "big_keys": st["big_keys"],
              "merge_ranges": st["merge_ranges"], "merge_keys": st["merge_keys"],
              "device_errors": st["device_errors"]}
    if args.trace_file:
        with open(args.trace_file, "w") as f:
            json.dump({"workload": args.workload, "trace": trace, "kernels": kernels,
                       "stats": st}, f, indent=1)

    cpu = None
    if not args.no_cpu:
        sample_n = min(n, 1 << args.cpu_sample_log2)
        single_n = min(n, 1 << args.cpu_single_log2)
        print("bench: timing the oracle on %d keys (%d threads) and %d keys (1 thread)"
              % (sample_n, host_threads(), single_n), file=sys.stderr, flush=True)
        cpu = cpu_baseline(keys, kt, vals, sample_n, single_n, args.cpu_runs)

    value = n / (ms_per_step * 1e-3) / 1e9
    line = {
        "metric": "GKeys/s & % HBM roofline (uint64, n=2^28); batched/served keys/s + p50/p99",
        "value": round(value, 3),
        "unit": "GKeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "step_ms": step_stats,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {W.KEY_U64: "u64", W.KEY_U32: "u32", W.KEY_F32: "f32"}[kt] + ("+u32" if pay else ""),
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "distribution": dist,
                   "key": {W.KEY_U64: "uint64", W.KEY_U32: "uint32", W.KEY_F32: "float32"}[kt],
                   "payload": "uint32" if pay else None, "params": pkw},
        "roofline": roof,
        "passes": passes,
        "copy_ceiling": ceiling,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "levels": levels,
        "leaves": leaves,
        "verified": verified,
    }
    print(json.dumps(line))
    return 0


def copy_ceiling(api):
    """The practical HBM ceiling: the library's plain streaming copy of 2 GiB
    (4 GiB moved), best of five, with torch's copy kernel beside it."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.int64, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    nbytes = src.numel() * src.element_size()
    stream = torch.cuda.current_stream()
    from paper_1410_6754_amd._lib import check, lib

    def own():
        check(lib().ams_device_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream))

    def best_of(fn):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        return best

    ms_own = best_of(own)
    ok = bool(torch.equal(dst, src))
    dst.zero_()
    ms_torch = best_of(lambda: dst.copy_(src))
    del src, dst
    torch.cuda.empty_cache()
    moved = 2 * nbytes
    gbs = moved / (ms_own * 1e-3) / 1e9
    gbt = moved / (ms_torch * 1e-3) / 1e9
    return {"kernel": "ams_device_copy of 2 GiB (16 KiB per workgroup, 8 loads of 16 B per lane in flight)",
            "bytes_moved": moved, "ms": round(ms_own, 4), "GB_per_s": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "copy_verified": ok,
            "torch_copy_GB_per_s": round(gbt, 1)}


def pass_table(trace, st, w: int, kw: int, steps: int, ceiling_gbs: float):
    """Every HBM pass that had work, against the peak and the copy ceiling.

    Level l's passes touch only the keys of its subproblems (st["keys"][l]):
    keys placed in final children at earlier levels have dropped out, and a
    level without subproblems launches its kernels on empty lists, which are
    left out.  Count reads each key once (w_key bytes), the scatter reads and
    writes it (2w), the base case reads and writes the keys of its leaves
    (oversized leaves are first partitioned once more, a pass of their own).
    Returns (passes, per-kernel sums over the launches with work)."""
    by_name = {e["name"]: e for e in trace}
    passes = {}
    alg = {}

    def add(kernel, name, keys, per_key):
        e = by_name.get(name)
        if e is None or keys == 0:
            return None
        ms = e["total_ms"] / e["launches"]
        b = per_key * keys
        gbs = b / (ms * 1e-3) / 1e9
        passes[name] = {"avg_launch_ms": round(ms, 4), "keys": keys,
                        "algorithmic_bytes_per_launch": b, "GB_per_s": round(gbs, 1),
                        "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                        "frac_of_copy": round(gbs / ceiling_gbs, 4)}
        a = alg.setdefault(kernel, {"bytes": 0, "ms": 0.0, "launches": 0})
        a["bytes"] += b * e["launches"]
        a["ms"] += e["total_ms"]
        a["launches"] += e["launches"]
        return ms

    for l in range(st["levels"]):
        keys = st["keys"][l]
        mc = add("count", "count.L%d" % l, keys, kw)
        ms = add("scatter", "scatter.L%d" % l, keys, 2 * w)
        if mc is not None and ms is not None:
            # the level as a whole: 2w algorithmic bytes per key (read and
            # write), 3w moved by this implementation (count reads once more)
            lm = mc + ms
            gbs = 2 * w * keys / (lm * 1e-3) / 1e9
            passes["level.L%d" % l] = {
                "ms": round(lm, 4), "keys": keys, "algorithmic_bytes": 2 * w * keys,
                "implementation_bytes": (kw + 2 * w) * keys, "GB_per_s": round(gbs, 1),
                "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                "implementation_GB_per_s": round((kw + 2 * w) * keys / (lm * 1e-3) / 1e9, 1)}
    # oversized leaves: one more partition (a count read and a scatter, 2w
    # algorithmic bytes per key like a level's pass); their pieces are then
    # sorted by the base case with the other leaves
    add("big_part", "big_part", st["big_keys"], 2 * w)
    add("finish", "finish", st["leaf_keys"] + st["copy_keys"] + st["big_keys"], 2 * w)
    return passes, alg


def verify_against_device_sort(kt: int, d_keys, d_out, d_vout) -> bool:
    """The sort's output equals torch's device sort of the same input, bit for
    bit (keys mapped to signed integers of the same order; for pairs the
    stable sort's indices are the expected payload, which is 0..n-1)."""
    import torch
    if kt == W.KEY_U64:
        o = d_keys.view(torch.int64) ^ torch.iinfo(torch.int64).min
    elif kt == W.KEY_U32:
        o = d_keys.view(torch.int32) ^ torch.iinfo(torch.int32).min
    else:
        b = d_keys.view(torch.int32)
        o = torch.where(b >= 0, b, (~b) ^ torch.iinfo(torch.int32).min)
    sv, si = torch.sort(o, stable=True)
    del sv
    want = d_keys.view(o.dtype)[si]
    ok = bool(torch.equal(want, d_out.view(o.dtype)))
    if d_vout is not None:
        ok = ok and bool(torch.equal(si.to(torch.int64), d_vout.to(torch.int64)))
    del si, want, o
    torch.cuda.empty_cache()
    return ok


def _log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def verify_batch_against_device_sort(d_keys, d_out, offs) -> bool:
    """Every segment [offs[i], offs[i+1]) of d_out (uint64 keys) equals
    torch's device sort of that segment of d_keys: a stable sort by key, then
    a stable sort by segment, over runs of whole segments of at most 2^28
    keys."""
    import torch
    ok = True
    num = len(offs) - 1
    i = 0
    while i < num:
        j = i + 1
        while j < num and int(offs[j + 1]) - int(offs[i]) <= (1 << 28):
            j += 1
        a, b = int(offs[i]), int(offs[j])
        k = d_keys[a:b].view(torch.int64)
        _, i1 = torch.sort(k ^ torch.iinfo(torch.int64).min, stable=True)
        sz = torch.from_numpy((offs[i + 1:j + 1] - offs[i:j]).astype(np.int64)).to(k.device)
        seg = torch.repeat_interleave(torch.arange(j - i, dtype=torch.int32, device=k.device), sz)
        _, i2 = torch.sort(seg[i1], stable=True)
        ok = ok and bool(torch.equal(k[i1[i2]], d_out[a:b].view(torch.int64)))
        del i1, i2, seg, sz
        i = j
    torch.cuda.empty_cache()
    return ok


def _bits(t):
    """Signed-integer view of the same bits (for exact comparisons)."""
    import torch
    return t.view(torch.int64 if t.element_size() == 8 else torch.int32)


def bench_rlm(args) -> int:
    """RLM-sort of the same keys as the sample-sort workloads: tile sort, then
    per level multisequence selection and a merge pass.  The HBM passes are
    the tile sort and one merge per level, each reading and writing every
    key once (2w bytes per key); the selection is latency-bound."""
    import torch

    from paper_1410_6754_amd import api

    n, kt, dist, pkw, cfg = RLM_WORKLOADS[args.workload]
    if args.params:
        pkw = dict(pkw, **json.loads(args.params))
    w = key_bytes(kt)
    _log("generating %s (n=%d)" % (args.workload, n))
    keys = W.keys(kt, n, W.rng_for(cfg), dist)
    dev = torch.device("cuda:0")
    d_keys = torch.from_numpy(keys).to(dev)
    d_out = torch.empty_like(d_keys)
    params = api.rlm_params(**pkw)
    ws = api.alloc_workspace(api.rlm_workspace_bytes(kt, n, params), dev)
    stream = torch.cuda.current_stream()

    def step():
        api.rlm_sort_keys(d_keys, d_out, params=params, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    api.trace_start()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev0.record(stream)
    marks[0].record(stream)
    for i in range(args.steps):
        step()
        marks[i + 1].record(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    trace = api.trace_stop()
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    steps_ms = np.array([marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps)])
    verified = verify_against_device_sort(kt, d_keys, d_out, None)
    _log("%.3f ms/step; output %s the device reference sort"
         % (ms_per_step, "matches" if verified else "DIFFERS FROM"))
    ceiling = copy_ceiling(api)
    per = {}
    for e in trace:
        base = e["name"].split(".")[0]
        d = per.setdefault(base, {"launches": 0, "total_ms": 0.0})
        d["launches"] += e["launches"]
        d["total_ms"] += e["total_ms"]
    kernels = {k: {"launches": v["launches"], "avg_ms": round(v["total_ms"] / v["launches"], 4),
                   "share": round(v["total_ms"] / sum(x["total_ms"] for x in per.values()), 4)}
               for k, v in sorted(per.items(), key=lambda kv: -kv[1]["total_ms"])}
    passes = {}
    for e in trace:
        if e["name"] == "tile_sort" or e["name"].startswith("rlm_merge"):
            ms = e["total_ms"] / e["launches"]
            gbs = 2 * w * n / (ms * 1e-3) / 1e9
            passes[e["name"]] = {"avg_launch_ms": round(ms, 4), "keys": n,
                                 "algorithmic_bytes_per_launch": 2 * w * n,
                                 "GB_per_s": round(gbs, 1),
                                 "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                                 "frac_of_copy": round(gbs / ceiling["GB_per_s"], 4)}
    merge = per.get("rlm_merge")
    if merge:
        am = merge["total_ms"] / merge["launches"]
        achieved = 2 * w * n / (am * 1e-3) / 1e9
        roof = {"kernel": "rlm_merge", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic("rlm_merge", args.workload, RLM_SOURCES),
                "algorithmic_bytes_per_launch": 2 * w * n, "avg_launch_ms": round(am, 4)}
    else:
        roof = None
    line = {
        "metric": "GKeys/s & % HBM roofline (uint64, n=2^28); batched/served keys/s + p50/p99",
        "value": round(n / (ms_per_step * 1e-3) / 1e9, 3),
        "unit": "GKeys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "step_ms": {"min": round(float(steps_ms.min()), 4),
                    "median": round(float(np.median(steps_ms)), 4),
                    "p90": round(float(np.percentile(steps_ms, 90)), 4)},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {W.KEY_U64: "u64", W.KEY_U32: "u32", W.KEY_F32: "f32"}[kt],
        "data": "synthetic",
        "config": {"workload": args.workload, "algorithm": "RLM-sort (Section 5)", "n": n,
                   "distribution": dist, "params": pkw},
        "roofline": roof, "passes": passes, "copy_ceiling": ceiling, "kernels": kernels,
        "per_level_ms": {e["name"]: round(e["total_ms"] / e["launches"], 4) for e in trace},
        "cpu_baseline": None, "verified": verified,
    }
    print(json.dumps(line))
    return 0


def bench_batch(args) -> int:
    """Configuration 4: thousands of independent uint64 sorts of uneven sizes,
    one persistent batched call against one call per instance on the same
    stream (both through the C ABI, same defaults, same output)."""
    import ctypes

    import torch

    from paper_1410_6754_amd import _lib as L
    from paper_1410_6754_amd import api

    rng = W.rng_for(SPECIAL[args.workload])
    sizes = W.batch_sizes(20000, rng, 8, 20)
    if args.workload == "batch_2^28":
        sizes = W.truncate_total(sizes, 1 << 28)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = int(offs[-1])
    _log("%s: %d segments, %d keys (2^%.2f); generating" % (args.workload, sizes.size, total,
                                                         np.log2(total)))
    keys = W.uniform_u64(total, rng)
    dev = torch.device("cuda:0")
    d_keys = torch.from_numpy(keys).to(dev)
    d_out = torch.empty_like(d_keys)
    stream = torch.cuda.current_stream()
    lib = L.lib()
    s_ptr = stream.cuda_stream

    d_offs = torch.from_numpy(offs.astype(np.int64)).to(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_batched(params):
        """ms per batched call (and host wall ms) with these parameters."""
        wsb = api.batch_workspace_bytes(W.KEY_U64, offs, params=params)
        ws = api.alloc_workspace(wsb, dev)

        def batched():
            api.sort_batch(d_keys, offs, out_keys=d_out, d_offsets=d_offs, params=params,
                           workspace=ws, stream=stream)

        for _ in range(args.warmup):
            batched()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            batched()
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        del ws
        return ev0.elapsed_time(ev1) / args.steps, wall * 1e3

    # the built-in defaults, then the autotuner's choice for this batch (the
    # reported value); both sort into d_out and must agree
    ms_d, _ = time_batched(None)
    _log("batched, default parameters: %.3f ms per batch" % ms_d)
    t0 = time.perf_counter()
    tuned, tuned_ms = api.autotune(d_keys, offs, stream=stream, max_trials=args.tune_trials)
    tune_s = time.perf_counter() - t0
    _log("autotuned in %.1f s: %s (%.3f ms)" % (tune_s, api.params_dict(tuned), tuned_ms))
    ms_b, wall_b = time_batched(tuned)
    _log("batched, tuned parameters: %.3f ms per batch (wall %.3f ms)" % (ms_b, wall_b))

    # verify: every segment equals torch's device sort of it, and sampled
    # segments equal numpy's sort
    ok = verify_batch_against_device_sort(d_keys, d_out, offs)
    _log("every segment equals the device reference sort: %s" % ok)
    for i in np.linspace(0, sizes.size - 1, 40).astype(int):
        a, b = int(offs[i]), int(offs[i + 1])
        ok = ok and np.array_equal(d_out[a:b].cpu().numpy(), np.sort(keys[a:b]))

    # one call per instance through the C ABI, one workspace sized for the largest
    d_out2 = torch.empty_like(d_keys)
    wsb1 = api.workspace_bytes(W.KEY_U64, int(sizes.max()))
    ws1 = api.alloc_workspace(wsb1, dev)
    kin, kout, wsp = d_keys.data_ptr(), d_out2.data_ptr(), ws1.data_ptr()
    fn = lib.ams_sort_keys
    offl = [int(x) for x in offs]

    def per_instance():
        for i in range(sizes.size):
            a = offl[i]
            rc = fn(W.KEY_U64, kin + 8 * a, kout + 8 * a, offl[i + 1] - a, wsp, wsb1, s_ptr, None)
            if rc != 0:
                L.check(rc)

    per_instance()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    per_instance()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_p = time.perf_counter() - t0
    ms_p = ev0.elapsed_time(ev1)
    same = bool(torch.equal(_bits(d_out), _bits(d_out2)))
    _log("per instance: %.3f ms (wall %.3f ms); identical output: %s" % (ms_p, wall_p * 1e3, same))

    value = total / (ms_b * 1e-3) / 1e9
    line = {
        "metric": "batched sort throughput, GKeys/s (one persistent launch sequence with autotuned "
                  "parameters vs one call per instance)",
        "value": round(value, 3), "unit": "GKeys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_b, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": args.workload, "segments": int(sizes.size), "keys": total,
                   "sizes": "floor(2^U), U ~ Uniform(8, 20)", "min_size": int(sizes.min()),
                   "max_size": int(sizes.max()), "median_size": int(np.median(sizes))},
        "tuned_params": {k: v for k, v in api.params_dict(tuned).items() if v},
        "autotune_s": round(tune_s, 2),
        "default_params": {"value": round(total / (ms_d * 1e-3) / 1e9, 3), "unit": "GKeys/s",
                           "ms": round(ms_d, 3)},
        "per_instance": {"value": round(total / (ms_p * 1e-3) / 1e9, 3), "unit": "GKeys/s",
                         "ms": round(ms_p, 3), "host_wall_ms": round(wall_p * 1e3, 3)},
        "speedup_vs_per_instance": round(ms_p / ms_b, 2),
        "verified": bool(ok and same),
    }
    print(json.dumps(line))
    return 0 if ok and same else 1


def bench_serving(args) -> int:
    """Configuration 5: a Poisson stream of sort requests (sizes floor(2^U),
    U ~ U(10, 24); 50% uint64, 25% uint32, 25% float32 N(0,1)) into the
    serving loop.  Capacity is measured closed-loop (every request queued at
    once); then the stream is offered at 50%, 80% and 95% of it.  Latency =
    completion observed by the server - scheduled arrival."""
    import torch

    from paper_1410_6754_amd.server import Server

    rng = W.rng_for(SPECIAL["serving"])
    nreq = args.requests
    _, sizes, kts = W.serving_stream(nreq, rng, 1.0, 10, 24)
    dev = torch.device("cuda:0")
    _log("serving: %d requests, %d keys; generating" % (nreq, int(sizes.sum())))
    reqs = []
    for n, kt in zip(sizes, kts):
        k = W.keys(int(kt), int(n), rng, "uniform")
        reqs.append(torch.from_numpy(k).to(dev))
    torch.cuda.synchronize()
    total = int(sizes.sum())
    mean_keys = total / nreq

    def run(rate):
        """rate None: closed loop.  Returns (latencies_us, span_s)."""
        with Server(streams=2, max_pending=nreq + 8) as srv:
            # one warm request of every type
            for kt in (W.KEY_U64, W.KEY_U32, W.KEY_F32):
                x = next(r for r, t in zip(reqs, kts) if int(t) == kt)
                tk = srv.submit(x)
                srv.wait(tk)
                srv.release(tk)
            if rate is None:
                arr = np.zeros(nreq)
            else:
                gaps = np.random.default_rng([W.BASE_SEED + 5, int(rate)]).exponential(1.0 / rate, nreq)
                arr = np.cumsum(gaps) - gaps[0]
            tickets, late = [], []
            t0 = time.perf_counter()
            for i in range(nreq):
                while time.perf_counter() - t0 < arr[i]:
                    pass
                late.append((time.perf_counter() - t0 - arr[i]) * 1e6)
                tickets.append(srv.submit(reqs[i]))
            lat, first, last = [], None, None
            for i, tk in enumerate(tickets):
                st = srv.wait(tk)
                if st["status"] != 0:
                    raise RuntimeError("request %d failed: %d" % (i, st["status"]))
                lat.append(st["t_done_us"] - st["t_submit_us"] + late[i])
                first = st["t_submit_us"] if first is None else min(first, st["t_submit_us"])
                last = st["t_done_us"] if last is None else max(last, st["t_done_us"])
                srv.release(tk)
            return np.array(lat), (last - first) * 1e-6

    lat_c, span_c = run(None)
    cap = total / span_c
    _log("capacity (closed loop): %.3f GKeys/s over %.3f s" % (cap / 1e9, span_c))
    points = []
    for rho in (0.5, 0.8, 0.95):
        rate = rho * cap / mean_keys
        lat, span = run(rate)
        points.append({"offered": rho, "requests_per_s": round(rate, 1),
                       "achieved_GKeys_s": round(total / span / 1e9, 3),
                       "p50_us": round(float(np.percentile(lat, 50)), 1),
                       "p99_us": round(float(np.percentile(lat, 99)), 1)})
        _log("offered %.2f: %s" % (rho, points[-1]))

    # every result equals torch's device sort of its request
    ok = True
    with Server(streams=2, max_pending=nreq + 8) as srv:
        tickets = [srv.submit(r) for r in reqs]
        for i, tk in enumerate(tickets):
            st = srv.wait(tk)
            got = srv.result(tk)
            ok = ok and st["status"] == 0 and verify_against_device_sort(int(kts[i]), reqs[i], got, None)
            srv.release(tk)
    _log("every served result equals the device reference sort: %s" % ok)
    line = {
        "metric": "served sort throughput at capacity, GKeys/s, with p50/p99 latency at 50/80/95% load",
        "value": round(cap / 1e9, 3), "unit": "GKeys/s", "n_gpus": 1, "steps": nreq, "warmup": 3,
        "ms_per_step": round(span_c * 1e3 / nreq, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64/u32/f32", "data": "synthetic",
        "config": {"workload": "serving", "requests": nreq, "keys": total,
                   "sizes": "floor(2^U), U ~ Uniform(10, 24)", "types": "50% u64, 25% u32, 25% f32"},
        "closed_loop": {"p50_us": round(float(np.percentile(lat_c, 50)), 1),
                        "p99_us": round(float(np.percentile(lat_c, 99)), 1)},
        "load_points": points,
        "verified": ok,
    }
    print(json.dumps(line))
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
