#!/usr/bin/env python3
"""Benchmark of the anonymized-network-sensing hot path on one MI355X.

Headline (default `--workload aggregate_2p30`): 2^30 packets in 8192 windows
of 2^17 (Zipf 1.2 over a pool of 2^22, with a scanner and a sink) union-added
into one hypersparse traffic matrix, reduced to its eight quantities. A step is
one batched, graph-captured call (ns_batch_stats with the aggregate as its only
output); inputs are resident in HBM before the timed region. The plain way to
the same output is timed beside it: every window's matrix built by its own
ns_build_matrix call, the windows union-added by a balanced tree of
ns_accumulate calls, and ns_stats of the root. The same batched call that also
returns every window's eight quantities is reported as `with_per_window`.

The smaller workloads (one 2^17 window; 64 windows of 2^17 with their
aggregate; 1024 uneven windows) run as `secondary` entries of the same line,
each batched against its plain per-window loop, unless --no-secondary.

Prints one JSON line. `--gpus N` with N > 1 is refused: this path runs on one
GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

# what each workload computes (its config row)
OUTPUTS = {
    "aggregate_2p30": {"per_window": False, "aggregate": True},
    "windows64": {"per_window": True, "aggregate": True},
    "uneven1024": {"per_window": True, "aggregate": False},
    "one_window": {"per_window": True, "aggregate": False},
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="aggregate_2p30", choices=sorted(OUTPUTS))
    p.add_argument("--plain-steps", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-secondary", action="store_true",
                   help="skip the smaller workloads' batched-vs-plain entries")
    p.add_argument("--no-with-per-window", action="store_true",
                   help="aggregate workloads: skip timing the call that also returns every "
                        "window's quantities")
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="target CPU time of the oracle baseline sample")
    p.add_argument("--serve-arrivals", type=int, default=11024,
                   help="serving leg: arrivals (the first --serve-warm are warm-up); 0 = skip")
    p.add_argument("--serve-warm", type=int, default=1024)
    p.add_argument("--serve-rate", type=float, default=2000.0)
    p.add_argument("--no-analysis", action="store_true",
                   help="skip timing ns_stats on the pre-built aggregate")
    p.add_argument("--no-stream", action="store_true",
                   help="skip the out-of-core leg (packets streamed from host memory)")
    p.add_argument("--stream-batch", type=int, default=0,
                   help="out-of-core leg: packets per sub-partition (0: packets / 64, "
                        "at least 2^21)")
    p.add_argument("--copy-calibration-mib", type=int, default=0,
                   help="first run a plain device copy of this many MiB (3 times), whose "
                        "memory counters calibrate the profiler's byte counts")
    return p.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def host_info() -> dict:
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = None
    return {"nproc": os.cpu_count(), "affinity_cpus": aff, "cpu_model": model}


def timed_loop(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / max(steps, 1)


class PlainPath:
    """The plain way to a workload's outputs, one library call per window:
    ns_build_matrix of every window into a pool laid out by packet offset
    (window w's matrix starts at its first packet's position), ns_stats of each
    window when per-window quantities are wanted, and for the aggregate a
    balanced tree of ns_accumulate union-adds (level l+1 node i = nodes 2i and
    2i+1 of level l, in the other pool, over their joint packet range; an
    unpaired last node is union-added with the empty matrix), then ns_stats of
    the root."""

    def __init__(self, ns, torch, src_t, dst_t, off_np, dev, per_window, aggregate, ws):
        self.ns, self.torch = ns, torch
        self.src, self.dst, self.off = src_t, dst_t, [int(x) for x in off_np]
        self.W, self.N = len(self.off) - 1, self.off[-1]
        self.per_window, self.aggregate = per_window, aggregate
        n = max(self.N, 1)
        self.pool = [(torch.empty(n, dtype=torch.int64, device=dev),
                      torch.empty(n, dtype=torch.int64, device=dev))]
        if aggregate:
            self.pool.append((torch.empty(n, dtype=torch.int64, device=dev),
                              torch.empty(n, dtype=torch.int64, device=dev)))
        big = max(b - a for a, b in zip(self.off[:-1], self.off[1:])) if self.W else 1
        self.ws_win = ns.Workspace(max(big, 1), 1, device=dev)
        self.ws = ws  # large enough for the root's statistics
        self.mws = ns.MergeWorkspace(self.N, self.N, device=dev)
        self.st_w = torch.zeros((max(self.W, 1), 8), dtype=torch.int64, device=dev)
        self.st_a = torch.zeros(8, dtype=torch.int64, device=dev)
        self.empty = ns.Matrix(0, device=dev)
        ns.build_matrix(src_t[:0], dst_t[:0], self.empty, self.ws_win)
        # the tree's levels: node = (pool index, first window, end window)
        self.levels = []
        nodes = [(0, w, w + 1) for w in range(self.W)]
        self.nnz = [torch.zeros(max(self.W, 1), dtype=torch.int64, device=dev)]
        while aggregate and len(nodes) > 1:
            nxt = []
            for i in range(0, len(nodes), 2):
                pair = nodes[i:i + 2]
                nxt.append((1 - nodes[i][0], pair[0][1], pair[-1][2]))
            self.levels.append((nodes, nxt))
            self.nnz.append(torch.zeros(len(nxt), dtype=torch.int64, device=dev))
            nodes = nxt
        self.root = nodes[0] if nodes else None

    def _matrix(self, level, i, node, packets):
        ns = self.ns
        p, a, b = node
        lo, hi = self.off[a], self.off[b]
        keys, counts = self.pool[p]
        cap = hi - lo
        return ns.Matrix.wrap(keys[lo:lo + max(cap, 1)], counts[lo:lo + max(cap, 1)],
                              self.nnz[level][i:i + 1], cap, packets)

    def step(self):
        ns = self.ns
        mats = []
        for w in range(self.W):
            a, b = self.off[w], self.off[w + 1]
            m = self._matrix(0, w, (0, w, w + 1), 0)
            ns.build_matrix(self.src[a:b], self.dst[a:b], m, self.ws_win)
            if self.per_window:
                ns.stats(m, self.st_w[w], self.ws_win)
            mats.append(m)
        if not self.aggregate:
            return
        for lvl, (nodes, nxt) in enumerate(self.levels):
            out = []
            for i, node in enumerate(nxt):
                a_m = mats[2 * i]
                b_m = mats[2 * i + 1] if 2 * i + 1 < len(mats) else self.empty
                c = self._matrix(lvl + 1, i, node, 0)
                ns.accumulate(a_m, b_m, 1, c, self.mws)
                out.append(c)
            mats = out
        if mats:
            ns.stats(mats[0], self.st_a, self.ws)


def bytes_model(N, W, got, got_agg, per_window, aggregate, cmin, bits, scan_items=8):
    """Bytes the design as built moves for one step, from the measured links,
    sources and destinations of each pipeline that runs:
      sort with look-back: 8 (histogram) + 8 x 16 (key passes)
      single segment of at least `cmin` keys (chunked, digits of `bits` bits,
        P = 64 / bits key passes): P x (8 + 16)
      run-length: 8 read + 24 per link (items + the per-window matrix, or the
        aggregate's keys and counts) + 16 per row head
      row maxima: 16 per row head
      columns: 8 per link (histogram; look-back only, and not for one segment
        of 2^24 to 2^31 keys with run-length tiles of 16 keys per thread,
        whose run-length pass counts the digits) + 4 x 16 per link (passes;
        chunked: 32 / bits passes of 8 + 16) + 8 per link (run reduce) + 16
        per column head, and 16 per column head for the maxima."""
    P, Pc = -(-64 // bits), -(-32 // bits)

    def pipe(n, links, rows, cols, chunked, segments):
        fused = (not chunked and segments == 1 and scan_items == 16
                 and (1 << 24) <= n < (1 << 31))
        b = (P * 24 if chunked else 8 + 8 * 16) * n
        b += 8 * n + 24 * links + 16 * rows + 16 * rows
        b += (Pc * 24 if chunked else (0 if fused else 8) + 4 * 16) * links + 8 * links + 32 * cols
        return b
    total = 0
    if per_window:
        total += pipe(N, int(got[:, 1].sum()), int(got[:, 2].sum()), int(got[:, 3].sum()),
                      W == 1 and N >= cmin, W)
    if aggregate:
        total += pipe(N, int(got_agg[1]), int(got_agg[2]), int(got_agg[3]), N >= cmin, 1)
    return total


def sort_model_bytes(N, links):
    """The sort-method model of the method's algorithmic bytes with byte digits
    (8 key passes, 4 column passes): M = 16 + 16*8 + r*(76 + 24*4) bytes per
    packet, r = links / packets."""
    r = links / max(N, 1)
    return (16 + 16 * 8 + r * (76 + 24 * 4)) * N


def kernel_source_sha256() -> str:
    """Hash of the HIP sources, to tell whether stored counter data still
    describes the kernels that run."""
    d = os.path.join(ROOT, "paper_2510_14050_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def _traffic_file():
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    return t if t.get("source_sha256") == kernel_source_sha256() else None


def profiled_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 memory-counter summary (FETCH_SIZE and WRITE_SIZE passes, each
    scaled by what it reads for a 1 GiB copy), or None when the summary is
    missing or was taken on other kernel sources."""
    t = _traffic_file()
    for e in (t or {}).get("entries", []):
        if e["workload"] == workload and e["kernel"] == kernel:
            return e["traffic_bytes_per_launch"]
    return None


def path_rates(workload, N, W, got, got_agg, ms_step, per_window, aggregate, cmin, bits,
               scan_items=8):
    """Whole-step rates: measured memory traffic (rocprofv3 FETCH_SIZE +
    WRITE_SIZE of every library kernel of one step, scaled by a 1 GiB copy;
    null unless taken on these sources), the model bytes of the design as
    built, the sort-method model of the method's algorithmic bytes, and the
    floor of reading every packet once, each divided by the step time."""
    t = _traffic_file()
    measured = (t or {}).get("step_traffic_bytes", {}).get(workload)
    sec = ms_step * 1e-3
    M = bytes_model(N, W, got, got_agg, per_window, aggregate, cmin, bits, scan_items)
    links = int(got_agg[1]) if aggregate else int(got[:, 1].sum())
    S = sort_model_bytes(N, links)
    F = 8 * N + 64 * (W if per_window else 1)
    out = {"step_ms": round(ms_step, 4), "peak_gbs": PEAK_HBM_GBS,
           "model_bytes": M, "model_bytes_per_packet": round(M / max(N, 1), 2),
           "model_gbs": round(M / sec / 1e9, 1),
           "model_frac": round(M / sec / 1e9 / PEAK_HBM_GBS, 4),
           "method_bytes": round(S), "method_bytes_per_packet": round(S / max(N, 1), 2),
           "method_gbs": round(S / sec / 1e9, 1),
           "method_frac": round(S / sec / 1e9 / PEAK_HBM_GBS, 4),
           "floor_bytes": F, "floor_gbs": round(F / sec / 1e9, 1),
           "measured_bytes": measured, "measured_gbs": None, "measured_frac": None}
    if measured:
        out["measured_gbs"] = round(measured / sec / 1e9, 1)
        out["measured_frac"] = round(measured / sec / 1e9 / PEAK_HBM_GBS, 4)
    return out


def radix_roofline(kt, N, W, links_windows, agg_nnz, sort_block, sort_items, workload,
                   per_window, aggregate, cmin, bits):
    """Roofline of the dominant kernel, the radix pass (key passes after the
    first, which reads packets and is timed apart, and the column passes).
    Two kernels implement it: the look-back pass (byte digits: 7 + 4 passes;
    k_pass1 on one segment of at least 2^28 keys, else k_pass) and the
    chunked pass (one segment of at least `cmin` keys, digits of `bits` bits:
    64 / bits - 1 + 32 / bits passes). Algorithmic bytes = one
    8-byte read + one 8-byte write per key or column item moved; the report
    covers whichever kernel took longer, and lists both."""
    from paper_2510_14050_amd import ns
    chunk_kernel = "k_pass_chunked" if bits == 8 else "k_pass_chunked_wide"
    # one segment of at least 2^28 keys takes the early-ranking pass
    single_only = not per_window or W == 1
    lb_kernel = "k_pass1" if single_only and N >= (1 << 28) else "k_pass"
    narrow = "true" if N <= (1 << 31) - 2 else "false"  # 32-bit look-back words
    fams = {
        "k_pass": {"kernel": f"ns::{lb_kernel}<{sort_block}, {sort_items}, false, {narrow}>",
                   "kinds": ("pass", "col_pass"), "items": 0},
        "k_pass_chunked": {"kernel": "ns::%s<%d, %d, false>" % ((chunk_kernel,) + ns.CHUNKED_SHAPE),
                           "kinds": ("pass_chunked", "col_pass_chunked"), "items": 0},
    }
    runs = []
    if per_window:
        runs.append((W == 1 and N >= cmin, links_windows))
    if aggregate and not (per_window and W == 1):
        runs.append((N >= cmin, agg_nnz))
    for chunked, links in runs:
        P, Pc = (-(-64 // bits), -(-32 // bits)) if chunked else (8, 4)
        fams["k_pass_chunked" if chunked else "k_pass"]["items"] += (P - 1) * N + Pc * links
    rows = {}
    for name, f in fams.items():
        ms = sum(kt.get(k, (0.0, 0))[0] for k in f["kinds"])
        n = sum(kt.get(k, (0.0, 0))[1] for k in f["kinds"])
        if not n:
            continue
        byts = 16.0 * f["items"]
        ach = byts / (ms * 1e-3) / 1e9
        rows[name] = {"kernel": f["kernel"], "achieved": round(ach, 1),
                      "frac": round(ach / PEAK_HBM_GBS, 4), "total_ms": round(ms, 4),
                      "launches": n, "avg_launch_ms": round(ms / n, 5),
                      "algorithmic_bytes_per_launch": round(byts / n),
                      "traffic": profiled_traffic(workload, f["kernel"])}
    if not rows:
        return None
    top = max(rows.values(), key=lambda r: r["total_ms"])
    return {"bound": "hbm", "achieved": top["achieved"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": top["frac"], "traffic": top["traffic"], "kernel": top["kernel"],
            "avg_launch_ms": top["avg_launch_ms"], "launches": top["launches"],
            "algorithmic_bytes_per_launch": top["algorithmic_bytes_per_launch"],
            "kernels": rows}


def run_workload(name, args, dev, primary):
    """Batched vs plain on one workload; with primary=True also the kernel
    breakdown, roofline, analysis, out-of-core and CPU-baseline legs."""
    import numpy as np
    import torch

    from paper_2510_14050_amd import ns, synth, tune

    outs = OUTPUTS[name]
    per_window, aggregate = outs["per_window"], outs["aggregate"]
    wl = synth.WORKLOADS[name]()
    W, N = wl.num_windows, wl.total_packets
    log(f"workload {wl.name}: {W} windows, {N} packets; generating on the device")
    src_t, dst_t = wl.device_concat(dev)
    off_np = wl.offsets
    off_t = torch.from_numpy(off_np).to(dev)
    ws = ns.Workspace(N, W, device=dev)
    out = torch.zeros((W, 8), dtype=torch.int64, device=dev)
    agg = ns.Matrix(N, device=dev) if aggregate else None
    agg_stats = torch.zeros(8, dtype=torch.int64, device=dev) if aggregate else None
    torch.cuda.synchronize()

    shape = tune.lookup(N, W, aggregate_only=aggregate and not per_window)
    sort_block = shape.sort_block if shape else 256
    sort_items = shape.sort_items if shape else 16
    # single segments of at least cmin keys take the chunked passes, on digits of `bits` bits
    cmin = shape.chunked_min if shape and shape.chunked_min else ns.CHUNKED_MIN_DEFAULT
    bits = shape.digit_bits if shape and shape.digit_bits else 8
    log(f"launch shape: radix {sort_block}x{sort_items}, scan 256x"
        f"{shape.scan_items if shape else 8}, digit bits {bits}, "
        f"chunked from {cmin if cmin < (1 << 63) else 'never'} "
        f"({'autotuned' if shape else 'default: no tuning cache entry'} for {tune._device_name()})")
    out_arg = out if per_window else None

    def step(graph=True):
        ns.batch_stats(src_t, dst_t, off_t, out_arg, ws, agg=agg, agg_stats=agg_stats,
                       tune=shape, graph=graph)

    steps = args.steps if primary else max(5, min(args.steps, 20))
    ms_step = timed_loop(torch, step, steps, args.warmup)
    value = N / (ms_step * 1e-3)
    log(f"batched: {ms_step:.3f} ms/step, {value:.4e} packets/s")
    got = ns.stats_numpy(out).copy()
    got_agg = ns.stats_numpy(agg_stats).copy() if aggregate else None
    agg_nnz = agg.nnz() if aggregate else 0
    res = {"workload": wl.name, "windows": W, "total_packets": N, "value": value,
           "unit": "packets/s", "ms_per_step": round(ms_step, 4), "steps": steps,
           "outputs": ("per-window 8 stats" if per_window else "") +
                      (" + " if per_window and aggregate else "") +
                      ("aggregate matrix + aggregate 8 stats" if aggregate else ""),
           "submission": "one HIP graph (ns_batch_stats)"}
    if aggregate:
        res["aggregate_links"] = agg_nnz

    # the same call with every window's quantities as well (aggregate workloads)
    if primary and aggregate and not per_window and not args.no_with_per_window:
        def step_all():
            ns.batch_stats(src_t, dst_t, off_t, out, ws, agg=agg, agg_stats=agg_stats,
                           tune=shape)
        ms_all = timed_loop(torch, step_all, max(3, steps // 2), 1)
        same = bool(np.array_equal(ns.stats_numpy(agg_stats), got_agg))
        got = ns.stats_numpy(out).copy()
        res["with_per_window"] = {"ms_per_step": round(ms_all, 4), "value": N / (ms_all * 1e-3),
                                  "aggregate_same": same,
                                  "what": "ns_batch_stats returning every window's 8 stats "
                                          "as well as the aggregate's"}
        log(f"with per-window quantities: {ms_all:.3f} ms/step")

    if primary:
        # --- per-kernel durations from HIP events (eager replay of the same step) ---
        ns.timing_reset()
        ns.timing_enable(True)
        step(graph=False)
        torch.cuda.synchronize()
        kt = ns.timing_read()
        ns.timing_enable(False)
        ns.timing_reset()
        links_windows = int(got[:, 1].sum())
        res["roofline"] = radix_roofline(kt, N, W, links_windows, agg_nnz, sort_block,
                                         sort_items, name, per_window, aggregate, cmin, bits)
        res["kernels_ms"] = {k: {"ms": round(v[0], 4), "launches": v[1]} for k, v in kt.items()}
        log("kernel breakdown (eager, ms):", json.dumps(res["kernels_ms"]))
        res["path"] = path_rates(name, N, W, got, got_agg, ms_step, per_window, aggregate, cmin,
                                 bits, shape.scan_items if shape else 8)

    if primary and aggregate and not args.no_analysis:
        res["analysis"] = analysis_leg(ns, torch, np, agg, ws, N, got_agg, args, dev)
    if primary and aggregate and not args.no_stream:
        res["out_of_core"] = stream_leg(args, ns, torch, src_t, dst_t, agg, ws, dev)

    # --- plain: one library call per window (and a union-add tree) ---
    if not args.no_plain:
        pp = PlainPath(ns, torch, src_t, dst_t, off_np, dev, per_window, aggregate, ws)
        plain_steps = args.plain_steps if primary else max(2, args.plain_steps)
        pms = timed_loop(torch, pp.step, plain_steps, 1)
        ok = True
        if per_window:
            ok = ok and bool(np.array_equal(ns.stats_numpy(pp.st_w)[:W], got))
        if aggregate:
            ok = ok and bool(np.array_equal(ns.stats_numpy(pp.st_a), got_agg))
        res["plain"] = {"value": N / (pms * 1e-3), "ms_per_step": round(pms, 4),
                        "steps": plain_steps, "bit_exact_vs_batched": ok,
                        "what": ("per-window ns_build_matrix" +
                                 (" + ns_stats" if per_window else "") +
                                 (" + balanced ns_accumulate tree + ns_stats of the root"
                                  if aggregate else "") + ", one call each, one stream")}
        res["batched_vs_plain"] = round(value / res["plain"]["value"], 2)
        log(f"plain: {pms:.3f} ms/step ({res['batched_vs_plain']}x slower than batched)")
        del pp
        torch.cuda.empty_cache()

    # --- oracle on the host: parity sample and CPU baseline ---
    if primary and not args.no_cpu_baseline:
        res["cpu_baseline"], res["bit_exact"] = cpu_leg(args, wl, src_t, dst_t, off_np, got,
                                                        got_agg, per_window, aggregate)
    elif not primary and not args.no_cpu_baseline:
        # parity of the secondary workload on a few windows
        import oracle
        src, dst = synth.as_u32(src_t), synth.as_u32(dst_t)
        ok = True
        for w in sorted({0, W // 2, W - 1}):
            a, b = int(off_np[w]), int(off_np[w + 1])
            ok = ok and bool(np.array_equal(got[w], oracle.stats(src[a:b], dst[a:b])))
        if aggregate and N <= (1 << 24):
            ok = ok and bool(np.array_equal(got_agg, oracle.stats(src, dst)))
        res["bit_exact_sampled"] = ok
    del src_t, dst_t, ws, out, agg
    ns.release_graphs()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def analysis_leg(ns, torch, np, agg, ws, N, got_agg, args, dev):
    """The eight quantities of the pre-built aggregate matrix (construction
    excluded, the shape of the paper's timed analysis), from the library's COO
    and from the same matrix as hypersparse CSR."""
    agg_nnz = agg.nnz()
    an_st = torch.zeros(8, dtype=torch.int64, device=dev)
    reps = max(3, min(20, args.steps))
    an_ms = timed_loop(torch, lambda: ns.stats(agg, an_st, ws), reps, 2)
    out = {"ms": round(an_ms, 4), "matrix_nnz": agg_nnz, "packets": N,
           "packets_per_s": N / (an_ms * 1e-3),
           "same_as_batched": bool(np.array_equal(ns.stats_numpy(an_st), got_agg)),
           "what": "ns_stats on the pre-built aggregate matrix (construction excluded)"}
    keys = agg.keys[:agg_nnz]
    rows_t, per_row = torch.unique_consecutive(keys >> 32, return_counts=True)
    row_ptr = torch.zeros(rows_t.numel() + 1, dtype=torch.int64, device=dev)
    row_ptr[1:] = torch.cumsum(per_row, 0)
    rows32 = rows_t.to(torch.int32)
    cols32 = (keys & 0xFFFFFFFF).to(torch.int32)
    vals = agg.counts[:agg_nnz]
    csr_ws = torch.empty(max(ns.stats_csr_workspace_size(agg_nnz), 256), dtype=torch.uint8,
                         device=dev)
    csr_st = torch.zeros(8, dtype=torch.int64, device=dev)
    csr_ms = timed_loop(torch, lambda: ns.stats_csr(rows32, row_ptr, cols32, vals, N, csr_st,
                                                    ws=csr_ws), reps, 2)
    out["csr_ms"] = round(csr_ms, 4)
    out["csr_rows"] = int(rows_t.numel())
    out["csr_same_as_batched"] = bool(np.array_equal(ns.stats_numpy(csr_st), got_agg))
    log(f"analysis of the pre-built aggregate: {an_ms:.3f} ms ({agg_nnz} links); "
        f"from CSR: {csr_ms:.3f} ms")
    del keys, rows_t, per_row, row_ptr, rows32, cols32, csr_ws
    return out


def cpu_leg(args, wl, src_t, dst_t, off_np, got, got_agg, per_window, aggregate):
    """The oracle as it stands, timed on the host on a bounded sample of the
    same workload: the first k windows (k grown until about --cpu-seconds of
    single-threaded work): their aggregate's matrix and eight quantities for
    aggregate workloads, each window's quantities otherwise. The sample also
    checks the batched results bit-exactly."""
    import numpy as np

    import oracle
    from paper_2510_14050_amd import synth
    W = wl.num_windows
    host = host_info()
    bit_exact = True
    if aggregate and not per_window:
        # the aggregate of the first k windows: a short run sizes k so that the
        # timed run takes about --cpu-seconds
        k0 = min(W, 16)
        n0 = int(off_np[k0])
        s0, d0 = synth.as_u32(src_t[:n0]), synth.as_u32(dst_t[:n0])
        c0 = time.perf_counter()
        oracle.stats(s0, d0)
        per_pk = (time.perf_counter() - c0) / max(n0, 1)
        want_n = args.cpu_seconds / max(per_pk, 1e-12) / 1.15  # n log n grows a little
        k = int(np.searchsorted(off_np, want_n, side="right")) - 1
        k = max(k0, min(W, k))
        sample_n = int(off_np[k])
        src = synth.as_u32(src_t[:sample_n])
        dst = synth.as_u32(dst_t[:sample_n])
        c0 = time.perf_counter()
        st = oracle.stats(src, dst)
        sample_t = time.perf_counter() - c0
        rate, sample_w = sample_n / sample_t, k
        if k == W:
            bit_exact = bool(np.array_equal(st, got_agg))
        # parity of the sampled windows' quantities comes from the GPU tests; the
        # sample here checks every window the per-window call produced
        if got is not None and got.any():
            for w in (0, W - 1):
                a, b = int(off_np[w]), int(off_np[w + 1])
                s_w, d_w = synth.as_u32(src_t[a:b]), synth.as_u32(dst_t[a:b])
                bit_exact = bit_exact and bool(np.array_equal(got[w], oracle.stats(s_w, d_w)))
        cpu = {"value": rate, "unit": "packets/s", "cores": 1, "kind": "oracle",
               "sample": f"aggregate of the first {sample_w} of {W} windows ({sample_n} "
                         f"packets): matrix and its 8 quantities by the std::sort route, "
                         f"single thread, {sample_t:.1f} s",
               "windows_sampled": sample_w, "host": host}
        log(f"oracle: {rate:.4e} packets/s on the aggregate of {sample_w} windows")
        return cpu, bit_exact
    # host copies of the packets the sample may use (not timed)
    lim = int(off_np[min(W, 512)])
    src = synth.as_u32(src_t[:lim])
    dst = synth.as_u32(dst_t[:lim])
    c0 = time.perf_counter()
    want = []
    w = 0
    while w < W and int(off_np[w + 1]) <= lim and (time.perf_counter() - c0) < args.cpu_seconds / 2:
        a, b = int(off_np[w]), int(off_np[w + 1])
        want.append(oracle.stats(src[a:b], dst[a:b]))
        w += 1
    sampled_w = w
    sample_pk = int(off_np[sampled_w])
    agg_want = None
    if aggregate:
        agg_want = oracle.stats(src[:sample_pk], dst[:sample_pk])
    c1 = time.perf_counter()
    cpu_rate = sample_pk / (c1 - c0)
    cpu = {"value": cpu_rate, "unit": "packets/s", "cores": 1, "kind": "oracle",
           "sample": f"{sampled_w} of {W} windows ({sample_pk} packets): per-window "
                     f"8 quantities" + (" + aggregate matrix of the sampled windows and "
                                        "its 8 quantities" if aggregate else "") +
                     f", std::sort route, single thread, {c1 - c0:.1f} s",
           "windows_sampled": sampled_w, "host": host}
    bit_exact = bool(np.array_equal(got[:sampled_w], np.array(want).reshape(-1, 8)))
    if aggregate and sampled_w == W:
        bit_exact = bit_exact and bool(np.array_equal(got_agg, agg_want))
    if sampled_w > 1:
        # the same sample window-parallel on the host cores (the oracle's C
        # calls release the GIL, so threads run them side by side)
        from concurrent.futures import ThreadPoolExecutor
        T = max(1, min(16, host["affinity_cpus"] or os.cpu_count() or 1))

        def one(w):
            a, b = int(off_np[w]), int(off_np[w + 1])
            return oracle.stats(src[a:b], dst[a:b])
        p0 = time.perf_counter()
        with ThreadPoolExecutor(T) as ex:
            fagg = ex.submit(oracle.stats, src[:sample_pk], dst[:sample_pk]) if aggregate else None
            par = list(ex.map(one, range(sampled_w)))
            par_agg = fagg.result() if fagg else None
        p1 = time.perf_counter()
        cpu["parallel"] = {"value": sample_pk / (p1 - p0), "unit": "packets/s", "cores": T,
                           "kind": "oracle", "sample": f"the same sample, windows" +
                           (" and the aggregate" if aggregate else "") +
                           f" spread over {T} threads, {p1 - p0:.1f} s",
                           "agrees": bool(np.array_equal(np.array(par), np.array(want))
                                          and (not aggregate or np.array_equal(par_agg, agg_want)))}
        log(f"oracle window-parallel ({T} threads): {sample_pk / (p1 - p0):.4e} packets/s")
    log(f"oracle: {cpu_rate:.4e} packets/s on {sampled_w} windows; bit-exact {bit_exact}")
    return cpu, bit_exact


def stream_leg(args, ns, torch, src_t, dst_t, agg, ws, dev):
    """Out-of-core build (batching of Sec. III-C): the same packets from pinned
    host memory, in sub-partitions, copied on a second stream while the
    previous one is built and union-added. Reported beside the host-to-device
    copy alone and the device-resident build alone."""
    N = src_t.numel()
    src_h, dst_h = src_t.cpu().pin_memory(), dst_t.cpu().pin_memory()
    links = agg.nnz()
    batch = args.stream_batch or max(1 << 21, N // 64)
    batch = min(batch, max(N, 1))
    # the first sub-partition is built in place in the output, so the
    # capacity covers it as well as the aggregate's links
    out = ns.Matrix(max(links, batch, 1), device=dev)
    sws = ns.StreamWorkspace(batch, out.capacity, device=dev)
    cs = torch.cuda.Stream(device=dev)
    reps = 3
    status_before = ns.device_status()  # reads and clears what earlier legs left
    ms = timed_loop(torch, lambda: ns.build_matrix_streamed(src_h, dst_h, out, sws,
                                                            copy_stream=cs), reps, 1)
    status = ns.device_status()
    nnz = out.nnz()
    keys_eq = nnz == links and bool(torch.equal(out.keys[:links], agg.keys[:links]))
    counts_eq = nnz == links and bool(torch.equal(out.counts[:links], agg.counts[:links]))
    same = status == 0 and keys_eq and counts_eq
    sd, dd = torch.empty_like(src_t), torch.empty_like(dst_t)

    def h2d():
        sd.copy_(src_h, non_blocking=True)
        dd.copy_(dst_h, non_blocking=True)
    h2d_ms = timed_loop(torch, h2d, reps, 1)
    dev_m = ns.Matrix(N, device=dev)
    build_ms = timed_loop(torch, lambda: ns.build_matrix(src_t, dst_t, dev_m, ws), reps, 1)
    res = {"batch_packets": batch, "sub_partitions": (N + batch - 1) // batch,
           "ms": round(ms, 4), "packets_per_s": N / (ms * 1e-3),
           "h2d_ms": round(h2d_ms, 4), "h2d_gbs": round(8 * N / (h2d_ms * 1e-3) / 1e9, 1),
           "device_resident_build_ms": round(build_ms, 4),
           "same_as_batched_aggregate": same,
           "check": {"status": status, "status_before": status_before, "nnz": nnz,
                     "nnz_batched": links, "keys_equal": keys_eq, "counts_equal": counts_eq},
           "what": "ns_build_matrix_streamed from pinned host memory (copies on a second stream)"}
    log(f"out-of-core build: {ms:.3f} ms for {N} packets in {res['sub_partitions']} "
        f"sub-partitions (copy alone {h2d_ms:.3f} ms, device-resident build {build_ms:.3f} ms)")
    del dev_m, sd, dd, sws, out, src_h, dst_h
    return res


def serve_leg(args, dev):
    """Serving workload: windows of 2^10..2^17 packets (Zipf 1.2, pool 2^22),
    Poisson arrivals, rolling aggregate over the last 1024 windows, stats per
    arrival; p50/p99 over the arrivals after the warm-up."""
    import numpy as np
    import torch

    from paper_2510_14050_amd import serve, synth
    n = args.serve_arrivals
    wl = synth.serving(num=n, rate=args.serve_rate)
    log(f"serving: generating {n} windows ({wl.total_packets} packets)")
    wins = []
    for w in range(n):
        s_t, d_t = wl.window(w, device=dev)
        wins.append((synth.as_u32(s_t), synth.as_u32(d_t)))
    torch.cuda.synchronize()
    srv = serve.Server(ring=1024, max_window=1 << 17, max_batch=16, budget_bytes=4 << 30,
                       device=dev)
    # warm the library (first launches) off the clock
    srv.run(wins[:8])
    rep = srv.run(wins, arrivals_s=wl.arrivals[:n] - wl.arrivals[0])
    lat = rep.latencies_ms()[args.serve_warm:]
    measured = rep.results[args.serve_warm:]
    pk = sum(r.packets for r in measured)
    span = (measured[-1].t_done - measured[0].t_arrival) if measured else 0.0
    # spot-check a few rolling snapshots against the oracle
    import oracle
    checks = []
    for k in (args.serve_warm, n - 1):
        lo = max(0, k - 1023)
        want = oracle.stats(np.concatenate([wins[j][0] for j in range(lo, k + 1)]),
                            np.concatenate([wins[j][1] for j in range(lo, k + 1)]))
        checks.append(bool(np.array_equal(rep.results[k].rolling_stats, want)))
    out = {
        "workload": wl.name, "arrivals": n, "warmup_arrivals": args.serve_warm,
        "offered_windows_per_s": args.serve_rate, "ring": 1024,
        "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
        "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
        "mean_ms": round(float(lat.mean()), 3) if lat.size else None,
        "packets_per_s": pk / span if span else None,
        "mean_batch": round(float(np.mean(rep.batches)), 2),
        "max_batch": int(max(rep.batches)), "max_in_flight": rep.max_in_flight,
        "compactions": rep.compactions,
        "rolling_spot_checks_bit_exact": checks,
    }
    # where a micro-batch's time goes on the device (event timestamps), from a
    # second, shorter run with timed events (kept out of the latencies above):
    # its build (copies in + ns_batch_stats) and its rolling chain
    del srv
    torch.cuda.empty_cache()
    tsrv = serve.Server(ring=1024, max_window=1 << 17, max_batch=16, budget_bytes=4 << 30,
                        device=dev, timing=True)
    m = min(n, 2 * args.serve_warm + 1024)
    trep = tsrv.run(wins[:m], arrivals_s=wl.arrivals[:m] - wl.arrivals[0])
    skip = len(trep.batches) // 2
    bsp = np.array([e - s for _, s, e in trep.build_spans[skip:]])
    rsp = np.array([e - s for _, s, e in trep.roll_spans[skip:]])
    del tsrv
    if bsp.size:
        out["device_ms"] = {"build_p50": round(float(np.percentile(bsp, 50)), 3),
                            "build_p99": round(float(np.percentile(bsp, 99)), 3),
                            "rolling_p50": round(float(np.percentile(rsp, 50)), 3),
                            "rolling_p99": round(float(np.percentile(rsp, 99)), 3)}
    log("serving:", json.dumps(out))
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this path runs on a single GPU; multi-GPU runs are not supported "
              "(windows would shard across GPUs and the aggregate by a hash of its rows and "
              "columns, but neither exchange is built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_14050_amd import ns

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ns.load()

    if args.copy_calibration_mib:
        n64 = args.copy_calibration_mib * (1 << 20) // 8
        a = torch.ones(n64, dtype=torch.int64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.copy_calibration_mib} MiB "
            f"(read {args.copy_calibration_mib} MiB + write {args.copy_calibration_mib} MiB each)")
        del a, b

    head = run_workload(args.workload, args, dev, primary=True)
    secondary = None
    if not args.no_secondary:
        secondary = {}
        for name in ("one_window", "windows64", "uneven1024"):
            if name != args.workload:
                secondary[name] = run_workload(name, args, dev, primary=False)
    serving = serve_leg(args, dev) if args.serve_arrivals > 0 else None

    line = {
        "metric": "packets/sec (8 stats, bit-exact) batched vs plain; p50/p99 window latency",
        "value": head["value"],
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": head["workload"], "windows": head["windows"],
                   "total_packets": head["total_packets"], "outputs": head["outputs"],
                   "submission": head["submission"]},
        "roofline": head.get("roofline"),
        "path": head.get("path"),
        "cpu_baseline": head.get("cpu_baseline"),
        "plain": head.get("plain"),
        "batched_vs_plain": head.get("batched_vs_plain"),
        "bit_exact": head.get("bit_exact"),
        "with_per_window": head.get("with_per_window"),
        "analysis": head.get("analysis"),
        "out_of_core": head.get("out_of_core"),
        "kernels_ms": head.get("kernels_ms"),
        "secondary": secondary,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
