#!/usr/bin/env python3
"""Benchmark of the anonymized-network-sensing hot path on one MI355X.

A step is one pass of the whole path over the 64-window workload: 64 windows
of 2^17 packets (sources Zipf 1.1, destinations Zipf 1.3, pool 2^20) ->
every window's traffic matrix and eight quantities, plus the union-added
aggregate matrix of all windows and its eight quantities, submitted as one
graph-captured batched call (ns_batch_stats). Inputs are resident in HBM
before the timed region. The same work done the plain way (per-window
ns_build_matrix + ns_stats launches and an ns_accumulate chain for the
aggregate) is timed beside it.

Prints one JSON line. `--gpus N` with N > 1 is refused: this path runs on one
GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="windows64",
                   choices=["windows64", "one_window", "uneven1024", "aggregate_2p30"])
    p.add_argument("--plain-steps", type=int, default=5)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0,
                   help="target CPU time of the oracle baseline sample")
    p.add_argument("--serve-arrivals", type=int, default=11024,
                   help="serving leg: arrivals (the first --serve-warm are warm-up); 0 = skip")
    p.add_argument("--serve-warm", type=int, default=1024)
    p.add_argument("--serve-rate", type=float, default=2000.0)
    p.add_argument("--no-analysis", action="store_true",
                   help="skip timing ns_stats on the pre-built aggregate")
    p.add_argument("--no-stream", action="store_true",
                   help="skip the out-of-core leg (packets streamed from host memory)")
    p.add_argument("--stream-batch", type=int, default=1 << 21,
                   help="out-of-core leg: packets per sub-partition")
    p.add_argument("--copy-calibration-mib", type=int, default=0,
                   help="first run a plain device copy of this many MiB (3 times), whose "
                        "memory counters calibrate the profiler's byte counts")
    return p.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this path runs on a single GPU; multi-GPU runs are not supported "
              "(windows would shard across GPUs and the aggregate by a hash of its rows and "
              "columns, but neither exchange is built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2510_14050_amd import ns, synth, tune

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

    wl = synth.WORKLOADS[args.workload]()
    W, N = wl.num_windows, wl.total_packets
    log(f"workload {wl.name}: {W} windows, {N} packets; generating on the device")
    src_t, dst_t = wl.device_concat(dev)
    off_np = wl.offsets
    off_t = torch.from_numpy(off_np).to(dev)
    ws = ns.Workspace(N, W, device=dev)
    out = torch.zeros((W, 8), dtype=torch.int64, device=dev)
    agg = ns.Matrix(N, device=dev)
    agg_stats = torch.zeros(8, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()

    shape = tune.lookup(N, W)  # autotuned launch shape for this size class, if cached
    sort_block = shape.sort_block if shape else 256
    sort_items = shape.sort_items if shape else 16
    log(f"launch shape: radix {sort_block}x{sort_items}, scan 256x"
        f"{shape.scan_items if shape else 8} "
        f"({'autotuned' if shape else 'default: no tuning cache entry'} for {tune._device_name()})")

    def step():
        ns.batch_stats(src_t, dst_t, off_t, out, ws, agg=agg, agg_stats=agg_stats, tune=shape)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = N * args.steps / (t1 - t0)
    log(f"batched: {ms_step:.3f} ms/step, {value:.4e} packets/s")
    got = ns.stats_numpy(out).copy()
    got_agg = ns.stats_numpy(agg_stats).copy()
    agg_nnz = agg.nnz()

    # --- per-kernel durations from HIP events (eager replay of the same step) ---
    ns.timing_reset()
    ns.timing_enable(True)
    ns.batch_stats(src_t, dst_t, off_t, out, ws, agg=agg, agg_stats=agg_stats, tune=shape,
                   graph=False)
    torch.cuda.synchronize()
    kt = ns.timing_read()
    ns.timing_enable(False)
    ns.timing_reset()
    links_windows = int(got[:, 1].sum())
    roof = radix_roofline(kt, N, W, links_windows, agg_nnz, sort_block, sort_items, args.workload)
    breakdown = {k: {"ms": round(v[0], 4), "launches": v[1]} for k, v in kt.items()}
    log("kernel breakdown (eager, ms):", json.dumps(breakdown))

    # --- analysis only: the eight quantities of the pre-built aggregate matrix
    # (construction excluded, the shape of the paper's timed analysis) ---
    analysis = None
    if not args.no_analysis:
        an_st = torch.zeros(8, dtype=torch.int64, device=dev)
        for _ in range(2):
            ns.stats(agg, an_st, ws)
        torch.cuda.synchronize()
        reps = max(3, min(50, args.steps))
        a0 = time.perf_counter()
        for _ in range(reps):
            ns.stats(agg, an_st, ws)
        torch.cuda.synchronize()
        an_ms = (time.perf_counter() - a0) * 1e3 / reps
        analysis = {"ms": round(an_ms, 4), "matrix_nnz": agg_nnz, "packets": N,
                    "packets_per_s": N / (an_ms * 1e-3),
                    "same_as_batched": bool(np.array_equal(ns.stats_numpy(an_st), got_agg)),
                    "what": "ns_stats on the pre-built aggregate matrix (construction excluded)"}
        # the same matrix as hypersparse CSR (the form of the challenge's files),
        # converted on the device before timing
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
        for _ in range(2):
            ns.stats_csr(rows32, row_ptr, cols32, vals, N, csr_st, ws=csr_ws)
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        for _ in range(reps):
            ns.stats_csr(rows32, row_ptr, cols32, vals, N, csr_st, ws=csr_ws)
        torch.cuda.synchronize()
        csr_ms = (time.perf_counter() - a0) * 1e3 / reps
        analysis["csr_ms"] = round(csr_ms, 4)
        analysis["csr_rows"] = int(rows_t.numel())
        analysis["csr_same_as_batched"] = bool(np.array_equal(ns.stats_numpy(csr_st), got_agg))
        del keys, rows_t, per_row, row_ptr, rows32, cols32, csr_ws
        log(f"analysis of the pre-built aggregate: {an_ms:.3f} ms ({agg_nnz} links); "
            f"from CSR: {csr_ms:.3f} ms")

    # --- out-of-core: the aggregate built from packets in host memory ---
    outofcore = None
    if not args.no_stream:
        outofcore = stream_leg(args, ns, torch, src_t, dst_t, agg, ws, dev)

    # --- plain per-window path ---
    plain = None
    if not args.no_plain:
        wins = [ns.Matrix(int(wl.sizes[w]), device=dev) for w in range(W)]
        accs = [ns.Matrix(N, device=dev), ns.Matrix(N, device=dev)]
        st_w = torch.zeros((W, 8), dtype=torch.int64, device=dev)
        st_a = torch.zeros(8, dtype=torch.int64, device=dev)
        empty = ns.Matrix(0, device=dev)
        ns.build_matrix(src_t[:0], dst_t[:0], empty, ws)

        def plain_step():
            cur = empty
            for w in range(W):
                a, b = int(off_np[w]), int(off_np[w + 1])
                ns.build_matrix(src_t[a:b], dst_t[a:b], wins[w], ws)
                ns.stats(wins[w], st_w[w], ws)
                nxt = accs[w & 1]
                ns.accumulate(cur, wins[w], 1, nxt, ws)
                cur = nxt
            ns.stats(cur, st_a, ws)

        plain_step()
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            plain_step()
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        plain_ms = (p1 - p0) * 1e3 / args.plain_steps
        plain = {"value": N / (plain_ms * 1e-3), "ms_per_step": round(plain_ms, 4),
                 "bit_exact_vs_batched": bool(np.array_equal(ns.stats_numpy(st_w), got)
                                              and np.array_equal(ns.stats_numpy(st_a), got_agg))}
        log(f"plain: {plain_ms:.3f} ms/step, {plain['value']:.4e} packets/s")

    # --- oracle on the host: parity and CPU baseline ---
    cpu = None
    bit_exact = None
    if not args.no_cpu_baseline:
        import oracle
        src = synth.as_u32(src_t)
        dst = synth.as_u32(dst_t)
        # bounded sample: whole windows (and the aggregate of the sampled windows)
        # until about --cpu-seconds of single-threaded oracle work
        c0 = time.perf_counter()
        done_pk, w = 0, 0
        want = np.zeros((W, 8), np.uint64)
        while w < W and (time.perf_counter() - c0) < args.cpu_seconds / 2:
            a, b = int(off_np[w]), int(off_np[w + 1])
            want[w] = oracle.stats(src[a:b], dst[a:b])
            done_pk += b - a
            w += 1
        sampled_w = w
        sample_pk = int(off_np[sampled_w])
        agg_want = oracle.stats(src[:sample_pk], dst[:sample_pk])
        done_pk += sample_pk
        c1 = time.perf_counter()
        # the sample processes sample_pk packets per window pass and per aggregate
        cpu_rate = sample_pk / (c1 - c0)
        cpu = {"value": cpu_rate, "unit": "packets/s", "cores": 1, "kind": "oracle",
               "sample": f"{sampled_w} of {W} windows ({sample_pk} packets): per-window "
                         f"8 quantities + aggregate matrix and its 8 quantities, "
                         f"std::sort route, single thread, {c1 - c0:.1f} s"}
        if sampled_w > 1:
            # the same sample window-parallel on the host cores (the oracle's C
            # calls release the GIL, so threads run them side by side)
            from concurrent.futures import ThreadPoolExecutor
            T = max(1, min(16, os.cpu_count() or 1))
            def one(w):
                a, b = int(off_np[w]), int(off_np[w + 1])
                return oracle.stats(src[a:b], dst[a:b])
            p0 = time.perf_counter()
            with ThreadPoolExecutor(T) as ex:
                fagg = ex.submit(oracle.stats, src[:sample_pk], dst[:sample_pk])
                par = list(ex.map(one, range(sampled_w)))
                par_agg = fagg.result()
            p1 = time.perf_counter()
            cpu["parallel"] = {"value": sample_pk / (p1 - p0), "unit": "packets/s", "cores": T,
                               "kind": "oracle", "sample": f"the same sample, windows and the "
                               f"aggregate spread over {T} threads, {p1 - p0:.1f} s",
                               "agrees": bool(np.array_equal(np.array(par), want[:sampled_w])
                                              and np.array_equal(par_agg, agg_want))}
            log(f"oracle window-parallel ({T} threads): {sample_pk / (p1 - p0):.4e} packets/s")
        bit_exact = bool(np.array_equal(got[:sampled_w], want[:sampled_w]))
        if sampled_w == W:
            bit_exact = bit_exact and bool(np.array_equal(got_agg, agg_want))
        log(f"oracle: {cpu_rate:.4e} packets/s on {sampled_w} windows; bit-exact {bit_exact}")

    serving = None
    if args.serve_arrivals > 0:
        serving = serve_leg(args, dev)

    line = {
        "metric": "packets/sec (8 stats, bit-exact) batched vs plain; p50/p99 window latency",
        "value": value,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": wl.name, "windows": W, "total_packets": N,
                   "outputs": "per-window 8 stats + aggregate matrix + aggregate 8 stats",
                   "submission": "one HIP graph (ns_batch_stats)"},
        "roofline": roof,
        "path": path_rates(args.workload, N, W, got, got_agg, ms_step),
        "cpu_baseline": cpu,
        "analysis": analysis,
        "out_of_core": outofcore,
        "plain": plain,
        "batched_vs_plain": round(value / plain["value"], 2) if plain else None,
        "bit_exact": bit_exact,
        "kernels_ms": breakdown,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


def kernel_source_sha256() -> str:
    """Hash of the HIP sources, to tell whether stored counter data still
    describes the kernels that run."""
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2510_14050_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 memory-counter summary (FETCH_SIZE and WRITE_SIZE passes, each
    scaled by what it reads for a 1 GiB copy), or None when the summary is
    missing or was taken on other kernel sources."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_sha256():
        return None
    for e in t.get("entries", []):
        if e["workload"] == workload and e["kernel"] == kernel:
            return e["traffic_bytes_per_launch"]
    return None


def model_bytes(N, W, got, got_agg):
    """Bytes the design as built moves for one step (per-window pipeline plus
    the aggregate pipeline), from the measured links, sources and destinations:
      multi-segment sort (look-back): 8 (histogram) + 8 x 16 (key passes)
      single segment >= CHUNKED_MIN_DEFAULT (chunked): 8 x (8 + 16)
      run-length: 8 read + 24 per link (items + the per-window matrix, or the
        aggregate's keys and counts) + 16 per row head
      row maxima: 16 per row head
      columns: 8 per link (histogram; look-back only) + 4 x 16 per link
        (passes; +8 each when chunked) + 8 per link (run reduce) + 16 per
        column head, and 16 per column head for the maxima."""
    from paper_2510_14050_amd import ns
    cmin = ns.CHUNKED_MIN_DEFAULT
    def pipe(n, links, rows, cols, chunked):
        b = (8 * 24 if chunked else 8 + 8 * 16) * n
        b += 8 * n + 24 * links + 16 * rows + 16 * rows
        b += (4 * 24 if chunked else 8 + 4 * 16) * links + 8 * links + 32 * cols
        return b
    win = pipe(N, int(got[:, 1].sum()), int(got[:, 2].sum()), int(got[:, 3].sum()),
               W == 1 and N >= cmin)
    agg = pipe(N, int(got_agg[1]), int(got_agg[2]), int(got_agg[3]), N >= cmin)
    return win + agg


def path_rates(workload, N, W, got, got_agg, ms_step):
    """Whole-step rates: measured memory traffic (rocprofv3 FETCH_SIZE +
    WRITE_SIZE of every library kernel of one step, scaled by a 1 GiB copy;
    null unless taken on these sources), the model bytes of the design, and
    the floor of reading every packet once, each divided by the step time."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic.json")
    measured = None
    try:
        with open(path) as f:
            t = json.load(f)
        if t.get("source_sha256") == kernel_source_sha256():
            measured = t.get("step_traffic_bytes", {}).get(workload)
    except (OSError, ValueError):
        pass
    sec = ms_step * 1e-3
    M = model_bytes(N, W, got, got_agg)
    F = 8 * N + 64 * W
    out = {"step_ms": round(ms_step, 4), "peak_gbs": PEAK_HBM_GBS,
           "model_bytes": M, "model_bytes_per_packet": round(M / max(N, 1), 2),
           "model_gbs": round(M / sec / 1e9, 1), "model_frac": round(M / sec / 1e9 / PEAK_HBM_GBS, 4),
           "floor_bytes": F, "floor_gbs": round(F / sec / 1e9, 1),
           "measured_bytes": measured, "measured_gbs": None, "measured_frac": None}
    if measured:
        out["measured_gbs"] = round(measured / sec / 1e9, 1)
        out["measured_frac"] = round(measured / sec / 1e9 / PEAK_HBM_GBS, 4)
    return out


def radix_roofline(kt, N, W, links_windows, agg_nnz, sort_block, sort_items, workload):
    """Roofline of the dominant kernel, the radix pass (key passes 2-8 and the
    four column passes; the first key pass reads packets and is timed apart).
    Two kernels implement it: k_pass (decoupled look-back, every multi-segment
    sort) and k_pass_chunked (one segment of at least CHUNKED_MIN_DEFAULT
    keys). Algorithmic bytes = one 8-byte read + one 8-byte write per key or
    column item moved; the report covers whichever kernel took longer, and
    lists both."""
    from paper_2510_14050_amd import ns
    cmin = ns.CHUNKED_MIN_DEFAULT
    fams = {
        "k_pass": {"kernel": f"ns::k_pass<{sort_block}, {sort_items}, false>",
                   "kinds": ("pass", "col_pass"), "items": 0},
        "k_pass_chunked": {"kernel": "ns::k_pass_chunked<%d, %d, false>" % ns.CHUNKED_SHAPE,
                           "kinds": ("pass_chunked", "col_pass_chunked"), "items": 0},
    }
    for chunked, links in ((W == 1 and N >= cmin, links_windows), (N >= cmin, agg_nnz)):
        fams["k_pass_chunked" if chunked else "k_pass"]["items"] += 7 * N + 4 * links
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


def stream_leg(args, ns, torch, src_t, dst_t, agg, ws, dev):
    """Out-of-core build (batching of Sec. III-C): the same packets from pinned
    host memory, in sub-partitions of --stream-batch packets, copied on a
    second stream while the previous one is built and union-added. Reported
    beside the host-to-device copy alone and the device-resident build alone."""
    N = src_t.numel()
    src_h, dst_h = src_t.cpu().pin_memory(), dst_t.cpu().pin_memory()
    links = agg.nnz()
    batch = min(args.stream_batch, max(N, 1))
    # the first sub-partition is built in place in the output, so the
    # capacity covers it as well as the aggregate's links
    out = ns.Matrix(max(links, batch, 1), device=dev)
    sws = ns.StreamWorkspace(batch, out.capacity, device=dev)
    cs = torch.cuda.Stream(device=dev)
    reps = 5

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    ms = timed(lambda: ns.build_matrix_streamed(src_h, dst_h, out, sws, copy_stream=cs))
    same = ns.device_status() == 0 and out.nnz() == links and \
        bool(torch.equal(out.keys[:links], agg.keys[:links])) and \
        bool(torch.equal(out.counts[:links], agg.counts[:links]))
    sd, dd = torch.empty_like(src_t), torch.empty_like(dst_t)

    def h2d():
        sd.copy_(src_h, non_blocking=True)
        dd.copy_(dst_h, non_blocking=True)
    h2d_ms = timed(h2d)
    dev_m = ns.Matrix(N, device=dev)
    build_ms = timed(lambda: ns.build_matrix(src_t, dst_t, dev_m, ws))
    res = {"batch_packets": batch, "sub_partitions": (N + batch - 1) // batch,
           "ms": round(ms, 4), "packets_per_s": N / (ms * 1e-3),
           "h2d_ms": round(h2d_ms, 4), "h2d_gbs": round(8 * N / (h2d_ms * 1e-3) / 1e9, 1),
           "device_resident_build_ms": round(build_ms, 4),
           "same_as_batched_aggregate": same,
           "what": "ns_build_matrix_streamed from pinned host memory (copies on a second stream)"}
    log(f"out-of-core build: {ms:.3f} ms for {N} packets in {res['sub_partitions']} "
        f"sub-partitions (copy alone {h2d_ms:.3f} ms, device-resident build {build_ms:.3f} ms)")
    del dev_m, sd, dd, sws, out
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
        "rolling_spot_checks_bit_exact": checks,
    }
    log("serving:", json.dumps(out))
    return out


if __name__ == "__main__":
    main()
