"""Autotuner for the batched path's launch configuration.

Times graph replays of ns_batch_stats on a given batch and caches the fastest
configuration in a JSON file keyed by device (ISA and CU count) and size class
(log2 of packets and of windows, with the suffix "_agg" for calls that compute
the aggregate alone). The sweep is staged, each stage keeping the winner of
the one before:
1. tile shapes: the radix tile (256/512 threads x 8/16 keys) and the
   run-length / run-reduce tile (256 x 8/16 positions);
2. bucket count of the single-segment sorts: byte digits (256 buckets, 8 key
   passes) or 11-bit digits (2048 buckets, 6 key passes), where the batch has
   a single segment large enough for the chunked passes;
3. the single-segment size from which the chunked passes are used (2^20, the
   default 2^24, or never), where the batch has a single segment in that range.
Lookups fall back to the nearest cached size class of the same device, then
to the library's defaults.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import ns

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.environ.get("NS_TUNE_CACHE", os.path.join(HERE, "tune_cache.json"))

SHAPES = [(256, 8, 8), (256, 16, 8), (512, 8, 8), (512, 16, 8), (512, 16, 16)]
DIGIT_BITS = (8, 11)
NEVER = (1 << 64) - 1
CHUNKED_MINS = (1 << 20, 1 << 24, NEVER)


def size_class(packets: int, windows: int, aggregate_only: bool = False) -> str:
    key = f"p{int(math.log2(max(packets, 1)))}_w{int(math.log2(max(windows, 1)))}"
    return key + "_agg" if aggregate_only else key


def _device_name() -> str:
    """Cache key of the current device: ISA and compute-unit count (the
    marketing name is not stable across tools that wrap the runtime)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{p.gcnArchName.split(':')[0]}/{p.multi_processor_count}CU"


def _load_cache() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _tuning(entry: dict):
    b, i, s = entry["shape"]
    return ns.tuning(sort_block=b, sort_items=i, scan_items=s,
                     digit_bits=entry.get("digit_bits", 8),
                     chunked_min=entry.get("chunked_min", 0))


def lookup(packets: int, windows: int, aggregate_only: bool = False):
    """Cached ns.Tuning for this size class on this device, or None. Calls
    that compute the aggregate alone have their own class (suffix "_agg"),
    and fall back to the class of the same size with per-window outputs."""
    cache = _load_cache().get(_device_name(), {})
    if not cache:
        return None
    key = size_class(packets, windows, aggregate_only)
    if key in cache:
        return _tuning(cache[key])
    key = size_class(packets, windows)
    plain = {k: v for k, v in cache.items() if not k.endswith("_agg")}
    if not plain:
        return None
    if key not in plain:
        def parts(k):
            p, w = k[1:].split("_w")
            return int(p), int(w)
        kp, kw = parts(key)
        key = min(plain, key=lambda k: abs(parts(k)[0] - kp) + abs(parts(k)[1] - kw))
    return _tuning(plain[key])


def _label(c: dict) -> str:
    cm = c["chunked_min"]
    cm_s = "never" if cm == NEVER else f"2^{int(math.log2(cm))}" if cm else "default"
    return f"{c['shape'][0]}x{c['shape'][1]}/{c['shape'][2]} d{c['digit_bits']} c{cm_s}"


def autotune(src, dst, offsets, ws, out, agg=None, agg_stats=None, reps: int = 10,
             shapes=SHAPES, save: bool = True) -> dict:
    """Time the staged sweep on this batch (out=None: the aggregate alone);
    cache and return the winning entry with every timing."""
    import torch
    W, N = offsets.numel() - 1, src.numel()
    aggregate_only = out is None
    times = {}

    def run(c: dict) -> float:
        t = _tuning(c)
        for _ in range(2):
            ns.batch_stats(src, dst, offsets, out, ws, agg=agg, agg_stats=agg_stats, tune=t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ns.batch_stats(src, dst, offsets, out, ws, agg=agg, agg_stats=agg_stats, tune=t)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        times[_label(c)] = ms
        ns.release_graphs()
        return ms

    best = {"shape": list(shapes[0]), "digit_bits": 8, "chunked_min": 0}
    # 1. tile shapes
    cands = [dict(best, shape=list(sh)) for sh in shapes]
    best = min(cands, key=run)
    # a single segment that the chunked passes sort: the aggregate, or one window
    single = N if (agg is not None or W == 1) else 0
    # 2. bucket count of the chunked single-segment sort
    if single >= (1 << 24):
        cands = [dict(best, digit_bits=d) for d in DIGIT_BITS]
        best = min(cands, key=lambda c: times.get(_label(c)) or run(c))
    # 3. the threshold of the chunked passes, where it changes the path
    if (1 << 20) <= single:
        cands = [dict(best, chunked_min=m) for m in CHUNKED_MINS]
        best = min(cands, key=lambda c: times.get(_label(c)) or run(c))
    entry = dict(best, ms=times, packets=N, windows=W, aggregate_only=aggregate_only)
    if save:
        cache = _load_cache()
        cache.setdefault(_device_name(), {})[size_class(N, W, aggregate_only)] = entry
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    return entry


# workload -> (per-window quantities, aggregate) of its configuration row,
# plus the 2^30 aggregate with every window's quantities as well
RUNS = {
    "one_window": [(True, False)],
    "windows64": [(True, True)],
    "uneven1024": [(True, False), (True, True)],
    "aggregate_2p30": [(False, True), (True, True)],
}


def main():
    """Tune the benchmark workloads and write the cache."""
    import argparse
    import sys

    import torch

    from . import synth
    p = argparse.ArgumentParser()
    p.add_argument("--workloads", default="one_window,windows64,uneven1024,aggregate_2p30")
    p.add_argument("--reps", type=int, default=10)
    args = p.parse_args()
    dev = torch.device("cuda:0")
    for name in args.workloads.split(","):
        wl = synth.WORKLOADS[name]()
        s, d = wl.device_concat(dev)
        off = torch.from_numpy(wl.offsets).to(dev)
        W, N = wl.num_windows, wl.total_packets
        ws = ns.Workspace(N, W, device=dev)
        for per_window, aggregate in RUNS[name]:
            out = torch.zeros((W, 8), dtype=torch.int64, device=dev) if per_window else None
            agg = ns.Matrix(N, device=dev) if aggregate else None
            agg_stats = torch.zeros(8, dtype=torch.int64, device=dev) if aggregate else None
            e = autotune(s, d, off, ws, out, agg, agg_stats, reps=args.reps)
            print(name, "per-window" if per_window else "", "aggregate" if aggregate else "",
                  json.dumps(e), file=sys.stderr, flush=True)
            del out, agg, agg_stats
            torch.cuda.empty_cache()
        del ws, s, d
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
