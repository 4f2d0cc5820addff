"""Serving loop: windows arrive over time; each gets its own eight quantities
and those of a device-resident rolling aggregate over the last `ring` windows.

Continuous batching, not a queue: arrivals that come while earlier ones are on
the GPU are admitted as soon as device memory for them is free (a staging
arena for their packets, a matrix arena for their traffic matrices), grouped
into one micro-batch and submitted as one batched call on the build stream.
The rolling chain (add the new window's matrix, subtract the window that left
the ring, reduce the aggregate) runs in arrival order on a second stream and
overlaps the next micro-batch's build. The rolling aggregate lives in device
hash tables (ns_rolling_update), so an arrival costs time proportional to the
two windows involved; mode="merge" keeps it as a sorted matrix updated by
union-add and subtract (ns_accumulate + ns_stats) instead, whose cost grows
with the aggregate. The rolling aggregate at arrival k is
over windows max(0, k-ring+1)..k by arrival sequence, whatever the batching.

Latency of an arrival = time its two result rows are on the host minus its
arrival time. All computation goes through the libns C ABI (ns_batch_stats,
replaying one captured graph per build slot and packet class, or
ns_batch_stats_eager with graphs=False; ns_rolling_update, ns_rolling_compact,
and in merge mode ns_accumulate and ns_stats); this module only moves bytes,
keeps lifetimes and keeps time.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import ns


class RingArena:
    """Circular allocator over [0, cap) for first-in first-out lifetimes."""

    def __init__(self, cap: int):
        self.cap = int(cap)
        self.live = collections.deque()  # (start, end) in allocation order
        self.head = 0

    def _place(self, n: int):
        n = max(int(n), 1)
        if n > self.cap:
            return None
        if not self.live:
            return 0
        oldest = self.live[0][0]
        if self.head > oldest:          # free: [head, cap) and [0, oldest)
            if self.head + n <= self.cap:
                return self.head
            return 0 if n <= oldest else None
        return self.head if self.head + n <= oldest else None   # free: [head, oldest)

    def can_alloc(self, n: int) -> bool:
        return self._place(n) is not None

    def alloc(self, n: int):
        start = self._place(n)
        if start is None:
            return None
        self.live.append((start, start + max(int(n), 1)))
        self.head = start + max(int(n), 1)
        return start

    def free_oldest(self):
        self.live.popleft()


@dataclass
class Result:
    seq: int
    packets: int
    window_stats: np.ndarray
    rolling_stats: np.ndarray
    t_arrival: float
    t_done: float
    batch: int

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass
class ServeReport:
    results: list
    batches: list = field(default_factory=list)      # windows per admitted micro-batch
    max_in_flight: int = 0                           # arrivals admitted, not yet on the host
    elapsed: float = 0.0
    compactions: int = 0
    build_spans: list = field(default_factory=list)  # (batch, t_start_ms, t_end_ms) on device
    roll_spans: list = field(default_factory=list)

    def latencies_ms(self) -> np.ndarray:
        return np.array([r.latency for r in self.results]) * 1e3

    def summary(self) -> dict:
        lat = self.latencies_ms()
        pk = sum(r.packets for r in self.results)
        return {
            "arrivals": len(self.results),
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_ms": float(lat.mean()) if lat.size else None,
            "max_ms": float(lat.max()) if lat.size else None,
            "packets_per_s": pk / self.elapsed if self.elapsed else None,
            "arrivals_per_s": len(self.results) / self.elapsed if self.elapsed else None,
            "mean_batch": float(np.mean(self.batches)) if self.batches else None,
            "max_batch": int(max(self.batches)) if self.batches else None,
            "max_in_flight": self.max_in_flight,
        }

    def device_overlap(self) -> int:
        """Number of micro-batch builds that ran on the device while an earlier
        batch's rolling chain was still running (from event timestamps)."""
        roll_end = {b: e for b, _, e in self.roll_spans}
        n = 0
        for b, s, _ in self.build_spans:
            if b - 1 in roll_end and s < roll_end[b - 1]:
                n += 1
        return n


class Server:
    """Rolling-aggregate network-sensing server on one GPU.

    ring          windows in the rolling aggregate (by arrival sequence)
    max_window    largest window accepted (packets)
    max_batch     most windows per micro-batch
    budget_bytes  device memory for window data: 16 B per packet for the window
                  matrices (held until the window leaves the ring) and 8 B per
                  packet of staging (held until its micro-batch is built). It
                  must hold ring + 2*max_batch windows of max_window packets.
    graphs        build micro-batches by replaying captured ns_batch_stats
                  graphs (two fixed slots of max_batch*max_window packets,
                  24 B per packet each, beside the budget), or launch them
                  eagerly
    """

    def __init__(self, ring: int = 1024, max_window: int = 1 << 17, max_batch: int = 16,
                 budget_bytes: int = 4 << 30, device="cuda", timing: bool = False,
                 mode: str = "hash", link_slots: int = 1 << 25, address_slots: int = 1 << 23,
                 graphs: bool = False):
        import torch
        self.torch = torch
        assert mode in ("hash", "merge")
        self.mode = mode
        self.ring, self.max_window, self.max_batch = ring, max_window, max_batch
        self.timing = timing
        self.dev = d = torch.device(device)
        mat_entries = (ring + 2 * max_batch) * max_window
        batch_pk = max_batch * max_window
        if budget_bytes < 16 * mat_entries + 8 * batch_pk:
            raise ValueError("memory budget cannot hold the ring at max_window plus a micro-batch")
        self.stage_cap = int(min((budget_bytes - 16 * mat_entries) // 8, 4 * batch_pk))
        self.mat_cap = int(mat_entries)
        self.stage_src = torch.empty(self.stage_cap, dtype=torch.int32, device=d)
        self.stage_dst = torch.empty(self.stage_cap, dtype=torch.int32, device=d)
        self.pin_src = torch.empty(self.stage_cap, dtype=torch.int32).pin_memory()
        self.pin_dst = torch.empty(self.stage_cap, dtype=torch.int32).pin_memory()
        self.mat_keys = torch.empty(self.mat_cap, dtype=torch.int64, device=d)
        self.mat_counts = torch.empty(self.mat_cap, dtype=torch.int64, device=d)
        self.ws_build = ns.Workspace(batch_pk, max_batch, device=d)
        self.s_build = torch.cuda.Stream(device=d)
        self.s_roll = torch.cuda.Stream(device=d)
        if mode == "merge":
            self.roll_cap = ring * max_window + max_window
            self.acc = [ns.Matrix(self.roll_cap, device=d) for _ in range(3)]
            self.ws_roll = ns.Workspace(self.roll_cap + max_window, 1, device=d)
        else:
            self.ws_roll = ns.Workspace(max_window, 1, device=d)
            self.states = [ns.RollingState(link_slots, address_slots, device=d, stream=self.s_roll)
                           for _ in range(2)]
            self.link_slots, self.address_slots = link_slots, address_slots
        self.slots = 8 * max_batch + 64     # result rows in flight (ring buffer by sequence)
        self.win_dev = torch.zeros((self.slots, 8), dtype=torch.int64, device=d)
        self.roll_dev = torch.zeros((self.slots, 8), dtype=torch.int64, device=d)
        self.win_host = torch.zeros((self.slots, 8), dtype=torch.int64).pin_memory()
        self.roll_host = torch.zeros((self.slots, 8), dtype=torch.int64).pin_memory()
        # slots taken in the rolling state's link / source / destination tables
        self.occ_dev = torch.zeros((self.slots, 3), dtype=torch.int64, device=d)
        self.occ_host = torch.zeros((self.slots, 3), dtype=torch.int64).pin_memory()
        self.bslots = self.slots            # per-batch offsets / nnz rows
        self.pin_off = torch.zeros((self.bslots, max_batch + 1), dtype=torch.int64).pin_memory()
        self.off_dev = torch.zeros((self.bslots, max_batch + 1), dtype=torch.int64, device=d)
        self.out_dev = torch.zeros((self.bslots, max_batch, 8), dtype=torch.int64, device=d)
        self.empty = ns.Matrix(0, device=d)
        with torch.cuda.stream(self.s_roll):
            ns.build_matrix(self.stage_src[:0], self.stage_dst[:0], self.empty, self.ws_roll)
        self.s_roll.synchronize()
        # Graph-replayed builds: a micro-batch is padded to max_batch windows
        # (empty ones) and its packet count rounded up to a power of two of at
        # least 2^10, and built in one of two fixed slots (inputs, window
        # matrices, link counts and quantities at fixed addresses), so each
        # (slot, packet class) pair replays one captured ns_batch_stats graph.
        # The slot's results are copied out on the build stream before the slot
        # is used again. All graphs are captured here, from empty batches.
        self.graphs = graphs
        if graphs:
            cap = batch_pk
            self.classes = []
            c = 1 << 10
            while c < cap:
                self.classes.append(c)
                c <<= 1
            self.classes.append(cap)
            self.gslots = []
            for _ in range(2):
                self.gslots.append({
                    "src": torch.zeros(cap, dtype=torch.int32, device=d),
                    "dst": torch.zeros(cap, dtype=torch.int32, device=d),
                    "off": torch.zeros(max_batch + 1, dtype=torch.int64, device=d),
                    "out": torch.zeros((max_batch, 8), dtype=torch.int64, device=d),
                    "win": ns.BatchMatrices(cap, max_batch, device=d),
                })
            with torch.cuda.stream(self.s_build):
                for g in self.gslots:
                    for c in self.classes:
                        ns.batch_stats(g["src"][:c], g["dst"][:c], g["off"], g["out"],
                                       self.ws_build, win=g["win"], graph=True)
            self.s_build.synchronize()

    def _packet_class(self, total: int) -> int:
        for c in self.classes:
            if total <= c:
                return c
        raise ValueError("micro-batch larger than max_batch * max_window")

    # -- one micro-batch ---------------------------------------------------------
    def _submit(self, st, batch, bidx):
        """batch: list of (seq, src, dst, t_arrival)."""
        torch = self.torch
        sizes = [b[1].size for b in batch]
        total = int(sum(sizes))
        W = len(batch)
        s0 = st.stage.alloc(total)
        m0 = st.mats.alloc(total)
        assert s0 is not None and m0 is not None
        off = np.zeros(W + 1, np.int64)
        np.cumsum(sizes, out=off[1:])
        ps, pd = self.pin_src.numpy(), self.pin_dst.numpy()
        for (_, s, d, _), o in zip(batch, off[:-1]):
            ps[s0 + o:s0 + o + s.size] = s.view(np.int32)
            pd[s0 + o:s0 + o + d.size] = d.view(np.int32)
        bs = bidx % self.bslots
        self.pin_off[bs, :W + 1] = torch.from_numpy(off)
        ev_b0 = torch.cuda.Event(enable_timing=True) if self.timing else None
        if self.graphs:
            self.pin_off[bs, W + 1:] = total  # padding windows are empty
        with torch.cuda.stream(self.s_build):
            if ev_b0 is not None:
                ev_b0.record(self.s_build)
            wm = ns.BatchMatrices(total, 0, device=self.dev,
                                  keys=self.mat_keys[m0:m0 + max(total, 1)],
                                  counts=self.mat_counts[m0:m0 + max(total, 1)])
            outs = self.out_dev[bs, :W]
            if self.graphs:
                g = self.gslots[bidx & 1]
                c = self._packet_class(total)
                g["src"][:total].copy_(self.pin_src[s0:s0 + total], non_blocking=True)
                g["dst"][:total].copy_(self.pin_dst[s0:s0 + total], non_blocking=True)
                g["off"].copy_(self.pin_off[bs], non_blocking=True)
                ns.batch_stats(g["src"][:c], g["dst"][:c], g["off"], g["out"], self.ws_build,
                               win=g["win"], graph=True)
                # out of the slot before its next use (same stream): the window
                # matrices into the matrix arena, link counts and quantities
                if total:
                    wm.keys[:total].copy_(g["win"].keys[:total])
                    wm.counts[:total].copy_(g["win"].counts[:total])
                outs.copy_(g["out"][:W])
                # per-window link counts live as long as the windows' matrices:
                # a fresh tensor, kept by the window views and marked as used by
                # the rolling stream so the allocator never recycles it early
                wm.nnz = g["win"].nnz[:max(W, 1)].clone()
            else:
                src = self.stage_src[s0:s0 + total]
                dst = self.stage_dst[s0:s0 + total]
                src.copy_(self.pin_src[s0:s0 + total], non_blocking=True)
                dst.copy_(self.pin_dst[s0:s0 + total], non_blocking=True)
                offs = self.off_dev[bs, :W + 1]
                offs.copy_(self.pin_off[bs, :W + 1], non_blocking=True)
                wm.nnz = torch.zeros(max(W, 1), dtype=torch.int64, device=self.dev)
                ns.batch_stats(src, dst, offs, outs, self.ws_build, win=wm, graph=False)
            wm.nnz.record_stream(self.s_roll)
            built = torch.cuda.Event(enable_timing=self.timing)
            built.record(self.s_build)
        st.stage_free.append(built)                 # staging reusable once built
        with torch.cuda.stream(self.s_roll):
            self.s_roll.wait_event(built)
            ev_r0 = torch.cuda.Event(enable_timing=True) if self.timing else None
            if ev_r0 is not None:
                ev_r0.record(self.s_roll)
            done = []
            for i, (seq, s, d, t_arr) in enumerate(batch):
                k = seq % self.slots
                self.win_dev[k].copy_(outs[i])
                win = wm.window(i, int(off[i]), sizes[i])
                st.views.append((seq, win, i == W - 1))
                old = None
                if len(st.views) > self.ring:
                    _, old, last_of_batch = st.views.popleft()
                if self.mode == "merge":
                    st.cur = self._accumulate(st, st.cur, win, 1)
                    if old is not None:
                        st.cur = self._accumulate(st, st.cur, old, -1)
                else:
                    ns.rolling_update(self.states[st.si], win, old, self.roll_dev[k])
                    self._maybe_compact(st, seq)
                    ns.rolling_occupancy(self.states[st.si], self.occ_dev[k])
                    self.occ_host[k].copy_(self.occ_dev[k], non_blocking=True)
                if old is not None and last_of_batch:  # its whole matrix region can go
                    ev = torch.cuda.Event()
                    ev.record(self.s_roll)
                    st.mat_free.append(ev)
                if self.mode == "merge":
                    ns.stats(st.cur, self.roll_dev[k], self.ws_roll)
                self.win_host[k].copy_(self.win_dev[k], non_blocking=True)
                self.roll_host[k].copy_(self.roll_dev[k], non_blocking=True)
                ev = torch.cuda.Event(enable_timing=self.timing)
                ev.record(self.s_roll)
                done.append(ev)
        if self.timing:
            st.timed.append((bidx, ev_b0, built, ev_r0, done[-1]))
        return done

    def _maybe_compact(self, st, seq: int):
        """Move the rolling state into the other buffer, dropping tombstones, once
        the slots taken in one of its tables (live entries plus tombstones, which
        the device counts) could pass 60% of it: the counts of the latest arrival
        the host has seen plus one per packet added since (a packet takes at most
        one new slot per table). Live entries are bounded the same way (and by
        the packets in the ring); only when that bound passes half a table are
        this update's exact counts read (one synchronisation) before the state is
        declared too small."""
        caps = (self.link_slots, self.address_slots, self.address_slots)
        kseq, used, live = st.known
        added = int(st.csum[seq + 1] - st.csum[kseq + 1]) if kseq >= 0 else int(st.csum[seq + 1])
        if all(u + added <= 0.6 * c for u, c in zip(used, caps)):
            return
        in_ring = int(st.csum[seq + 1] - st.csum[max(0, seq + 1 - self.ring)])
        live = tuple(min(lv + added, in_ring) for lv in live)
        if any(lv > 0.5 * c for lv, c in zip(live, caps)):
            # the bound is loose when the host has not seen a recent result:
            # wait for this update and take its exact counts
            self.s_roll.synchronize()
            rs = self.roll_dev[seq % self.slots].cpu()
            live = (int(rs[1]), int(rs[2]), int(rs[3]))
            if any(lv > 0.5 * c for lv, c in zip(live, caps)):
                raise RuntimeError("rolling aggregate outgrows its hash tables; "
                                   "raise the slot counts")
        nxt = 1 - st.si
        ns.rolling_compact(self.states[st.si], self.states[nxt])
        st.si = nxt
        with st.known_lock:  # the completer thread updates it too
            st.known = (seq, live, live)  # the new tables hold the live entries only
        st.compactions += 1

    def _accumulate(self, st, cur, win, sign):
        nxt = next(m for m in self.acc if m is not cur and m is not st.prev)
        ns.accumulate(cur, win, sign, nxt, self.ws_roll)
        st.prev = cur
        return nxt

    # -- the loop ----------------------------------------------------------------------
    def run(self, windows, arrivals_s=None) -> ServeReport:
        """Serve `windows` (list of (src, dst) uint32 arrays) arriving at the
        given times (s after the start; all at once when None)."""
        torch = self.torch
        n = len(windows)
        for s, d in windows:
            if s.size > self.max_window or s.size != d.size:
                raise ValueError("window larger than max_window or src/dst mismatch")

        class State:
            pass

        st = State()
        st.stage, st.mats = RingArena(self.stage_cap), RingArena(self.mat_cap)
        st.stage_free, st.mat_free = collections.deque(), collections.deque()
        st.views = collections.deque()
        st.cur, st.prev = self.empty, None
        st.timed = []
        st.si, st.compactions = 0, 0
        # latest counts on the host: (seq, slots taken per table, live links /
        # sources / destinations)
        st.known = (-1, (0, 0, 0), (0, 0, 0))
        st.known_lock = threading.Lock()
        st.sizes = np.array([w[0].size for w in windows], np.int64)
        st.csum = np.concatenate([[0], np.cumsum(st.sizes)])
        if self.mode == "hash":
            self.states[0].clear(self.s_roll)

        inbox = collections.deque()
        lock = threading.Lock()
        arrived = threading.Condition(lock)  # wakes the dispatcher on an arrival
        t_start = time.perf_counter()

        def feeder():
            for k in range(n):
                if arrivals_s is not None:
                    delay = t_start + float(arrivals_s[k]) - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                with arrived:
                    inbox.append((k, windows[k][0], windows[k][1], time.perf_counter()))
                    arrived.notify()

        results = [None] * n
        done_q = collections.deque()
        completed = [0]

        def completer():
            while completed[0] < n:
                if not done_q:
                    time.sleep(0.00005)
                    continue
                seq, t_arr, ev, bidx = done_q[0]
                ev.synchronize()
                t = time.perf_counter()
                k = seq % self.slots
                results[seq] = Result(seq, int(windows[seq][0].size),
                                      self.win_host[k].numpy().view(np.uint64).copy(),
                                      self.roll_host[k].numpy().view(np.uint64).copy(),
                                      t_arr, t, bidx)
                if self.mode == "hash":
                    u, rs = self.occ_host[k], results[seq].rolling_stats
                    with st.known_lock:  # never replace a later count (a compaction's)
                        if seq > st.known[0]:
                            st.known = (seq, (int(u[0]), int(u[1]), int(u[2])),
                                        (int(rs[1]), int(rs[2]), int(rs[3])))
                done_q.popleft()
                completed[0] += 1

        tf = threading.Thread(target=feeder, daemon=True)
        tc = threading.Thread(target=completer, daemon=True)
        tf.start()
        tc.start()
        report = ServeReport(results)
        submitted, bidx = 0, 0
        while submitted < n:
            while st.stage_free and st.stage_free[0].query():
                st.stage_free.popleft()
                st.stage.free_oldest()
            while st.mat_free and st.mat_free[0].query():
                st.mat_free.popleft()
                st.mats.free_oldest()
            with lock:
                ready = list(inbox)
            batch, total = [], 0
            for a in ready:
                t2 = total + a[1].size
                if (len(batch) == self.max_batch or t2 > self.max_batch * self.max_window
                        or submitted + len(batch) + 1 - completed[0] > self.slots - 1
                        or not st.stage.can_alloc(t2) or not st.mats.can_alloc(t2)):
                    break
                batch.append(a)
                total = t2
            if not batch:
                if ready:  # waiting for device memory or result slots
                    time.sleep(0.00005)
                else:
                    with arrived:
                        if not inbox:
                            arrived.wait(timeout=0.002)
                continue
            with lock:
                for _ in batch:
                    inbox.popleft()
            evs = self._submit(st, batch, bidx)
            report.batches.append(len(batch))
            for a, ev in zip(batch, evs):
                done_q.append((a[0], a[3], ev, bidx))
            submitted += len(batch)
            report.max_in_flight = max(report.max_in_flight, submitted - completed[0])
            bidx += 1
        tc.join()
        tf.join()
        torch.cuda.synchronize()
        report.elapsed = (max(r.t_done for r in results) - t_start) if n else 0.0
        report.compactions = st.compactions
        if self.timing and st.timed:
            t0 = st.timed[0][1]
            for b, e0, e1, r0, r1 in st.timed:
                report.build_spans.append((b, t0.elapsed_time(e0), t0.elapsed_time(e1)))
                report.roll_spans.append((b, t0.elapsed_time(r0), t0.elapsed_time(r1)))
        return report
