"""Autotuner for the batched path's launch shape.

Sweeps the radix tile (256/512 threads x 8/16 keys) and the run-length /
run-reduce tile (256 x 8/16 positions) on a given batch, timing graph replays of
ns_batch_stats, and caches the fastest shape in a JSON file keyed by device
name and size class (log2 of packets and of windows). Lookups fall back to
the nearest cached size class of the same device, then to the library's
defaults.
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


def size_class(packets: int, windows: int) -> str:
    return f"p{int(math.log2(max(packets, 1)))}_w{int(math.log2(max(windows, 1)))}"


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


def lookup(packets: int, windows: int, aggregate_only: bool = False):
    """Cached ns.Tuning for this size class on this device, or None. Calls
    that compute the aggregate alone have their own class (suffix "_agg"),
    and fall back to the class of the same size with per-window outputs."""
    cache = _load_cache().get(_device_name(), {})
    if not cache:
        return None
    key = size_class(packets, windows)
    if aggregate_only and key + "_agg" in cache:
        key = key + "_agg"
    cache = {k: v for k, v in cache.items() if not k.endswith("_agg")} if key not in cache \
        else cache
    if key not in cache:
        def dist(k):
            p, w = k[1:].split("_w")
            return abs(int(p) - int(key[1:].split("_w")[0])) + abs(int(w) - int(key.split("_w")[1]))
        key = min(cache, key=dist)
    b, i, s = cache[key]["shape"]
    return ns.tuning(sort_block=b, sort_items=i, digit_bits=8, scan_items=s)


def autotune(src, dst, offsets, ws, out, agg=None, agg_stats=None, reps: int = 10,
             shapes=SHAPES, save: bool = True) -> dict:
    """Time every shape on this batch; cache and return {"shape": best, "ms": {...}}."""
    import torch
    W, N = offsets.numel() - 1, src.numel()
    times = {}
    for shape in shapes:
        t = ns.tuning(sort_block=shape[0], sort_items=shape[1], digit_bits=8, scan_items=shape[2])
        for _ in range(2):
            ns.batch_stats(src, dst, offsets, out, ws, agg=agg, agg_stats=agg_stats, tune=t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ns.batch_stats(src, dst, offsets, out, ws, agg=agg, agg_stats=agg_stats, tune=t)
        torch.cuda.synchronize()
        times[f"{shape[0]}x{shape[1]}/{shape[2]}"] = (time.perf_counter() - t0) * 1e3 / reps
    best = min(shapes, key=lambda s: times[f"{s[0]}x{s[1]}/{s[2]}"])
    entry = {"shape": list(best), "ms": times, "packets": N, "windows": W}
    if save:
        cache = _load_cache()
        cache.setdefault(_device_name(), {})[size_class(N, W)] = entry
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    ns.release_graphs()
    return entry


def main():
    """Tune the benchmark workloads and write the cache."""
    import argparse
    import sys

    import torch

    from . import synth
    p = argparse.ArgumentParser()
    p.add_argument("--workloads", default="windows64,uneven1024,one_window,aggregate_2p30")
    p.add_argument("--reps", type=int, default=10)
    args = p.parse_args()
    dev = torch.device("cuda:0")
    for name in args.workloads.split(","):
        wl = synth.WORKLOADS[name]()
        s, d = wl.device_concat(dev)
        off = torch.from_numpy(wl.offsets).to(dev)
        W, N = wl.num_windows, wl.total_packets
        ws = ns.Workspace(N, W, device=dev)
        out = torch.zeros((W, 8), dtype=torch.int64, device=dev)
        agg = ns.Matrix(N, device=dev)
        agg_stats = torch.zeros(8, dtype=torch.int64, device=dev)
        e = autotune(s, d, off, ws, out, agg, agg_stats, reps=args.reps)
        print(name, json.dumps(e), file=sys.stderr, flush=True)
        del ws, out, agg, s, d
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
