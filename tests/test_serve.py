"""Serving loop: arena bookkeeping (CPU) and end-to-end results (GPU).

Every arrival's window quantities and rolling-aggregate quantities must equal
the oracle's, whatever the micro-batching and timing ("alone" = one window at
a time with nothing else in flight; "in the mix" = Poisson arrivals with
continuous batching and overlapping device work).
"""
import sys

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_2510_14050_amd import synth
from paper_2510_14050_amd.serve import RingArena


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@settings(max_examples=200, deadline=None)
@given(st.integers(16, 400), st.lists(st.tuples(st.booleans(), st.integers(1, 120)),
                                      max_size=200))
def test_ring_arena_fifo(cap, ops):
    """Live regions never overlap, stay in [0, cap), and frees are FIFO."""
    ar = RingArena(cap)
    live = []
    for is_alloc, n in ops:
        if is_alloc:
            can = ar.can_alloc(n)
            s = ar.alloc(n)
            assert (s is not None) == can
            if s is not None:
                assert 0 <= s and s + n <= cap
                for a, b in live:
                    assert s + n <= a or b <= s, "overlap"
                live.append((s, s + n))
        elif live:
            ar.free_oldest()
            live.pop(0)
    # with nothing live, the whole capacity is available
    while live:
        ar.free_oldest()
        live.pop(0)
    assert ar.can_alloc(cap)


def test_ring_arena_wraps():
    ar = RingArena(10)
    assert ar.alloc(4) == 0
    assert ar.alloc(4) == 4
    assert ar.alloc(4) is None      # only 2 left at the end, none at the front
    ar.free_oldest()
    assert ar.alloc(3) == 0         # wraps to the freed front
    assert ar.alloc(2) is None
    ar.free_oldest()
    assert ar.alloc(5) == 3


def small_windows(n_windows, seed=5, lo=8, hi=12):
    wl = synth.Workload("serve_t", seed, 1 << 12, 1.2, 1.2,
                        synth.log_uniform_sizes(seed, n_windows, lo, hi))
    return [wl.window(w) for w in range(n_windows)]


class _Stream:
    def __init__(self):
        self.syncs = 0

    def synchronize(self):
        self.syncs += 1


def _compaction_setup(monkeypatch, live, known, sizes):
    """A rolling state's host bookkeeping with the device parts stubbed on the
    CPU: 1000 link slots and 1000 address slots, a ring of 64 arrivals;
    `known` = (seq, slots taken, live counts) last seen on the host, `live` =
    this update's exact live counts."""
    import threading
    import types

    import torch

    from paper_2510_14050_amd import serve
    calls = []
    monkeypatch.setattr(serve.ns, "rolling_compact", lambda a, b: calls.append((a, b)))
    srv = types.SimpleNamespace(link_slots=1000, address_slots=1000, ring=64, slots=8,
                                s_roll=_Stream(), states=["state0", "state1"],
                                roll_dev=torch.zeros((8, 8), dtype=torch.int64))
    st = types.SimpleNamespace(si=0, compactions=0, known=known, known_lock=threading.Lock(),
                               sizes=np.array(sizes, np.int64))
    st.csum = np.concatenate([[0], np.cumsum(st.sizes)])
    seq = len(sizes) - 1
    srv.roll_dev[seq % 8, 1:4] = torch.tensor(live)
    return serve.Server._maybe_compact, srv, st, seq, calls


def test_compaction_waits_while_slots_taken_stay_low(monkeypatch):
    """Slots taken at the last count plus one per packet since stay below 60%
    of every table: nothing happens, however many packets went by."""
    fn, srv, st, seq, calls = _compaction_setup(monkeypatch, live=[0, 0, 0],
                                                known=(6, (300, 200, 100), (300, 200, 100)),
                                                sizes=[100] * 7 + [20])
    fn(srv, st, seq)
    assert srv.s_roll.syncs == 0 and calls == [] and st.compactions == 0


def test_compaction_reads_exact_counts_when_the_bound_is_loose(monkeypatch):
    """The host's last count is old (arrival 0): slots taken may pass 60%, and
    the live bound passes half a table although the update's exact live
    counts are small; the state is compacted after one synchronisation, not
    declared too small."""
    fn, srv, st, seq, calls = _compaction_setup(monkeypatch, live=[120, 80, 90],
                                                known=(0, (10, 10, 10), (10, 10, 10)),
                                                sizes=[10] + [100] * 7)
    fn(srv, st, seq)
    assert srv.s_roll.syncs == 1 and calls == [("state0", "state1")]
    assert st.si == 1 and st.compactions == 1
    assert st.known == (seq, (120, 80, 90), (120, 80, 90))


def test_compaction_keeps_the_bound_when_it_suffices(monkeypatch):
    """A recent count: slots taken may pass 60% of the link table, live entries
    stay below half of every table; compacted without synchronisation."""
    fn, srv, st, seq, calls = _compaction_setup(monkeypatch, live=[0, 0, 0],
                                                known=(6, (590, 200, 100), (300, 200, 100)),
                                                sizes=[100] * 7 + [20])
    fn(srv, st, seq)
    assert srv.s_roll.syncs == 0 and calls == [("state0", "state1")]
    assert st.known == (seq, (320, 220, 120), (320, 220, 120))


def test_compaction_refuses_a_state_that_is_too_small(monkeypatch):
    """Exact live counts past half a table raise."""
    fn, srv, st, seq, calls = _compaction_setup(monkeypatch, live=[700, 10, 10],
                                                known=(0, (10, 10, 10), (10, 10, 10)),
                                                sizes=[10] + [100] * 7)
    with pytest.raises(RuntimeError, match="outgrows"):
        fn(srv, st, seq)
    assert srv.s_roll.syncs == 1 and not calls


def rolling_want(windows, ring):
    out = []
    for k in range(len(windows)):
        lo = max(0, k - ring + 1)
        s = np.concatenate([windows[j][0] for j in range(lo, k + 1)])
        d = np.concatenate([windows[j][1] for j in range(lo, k + 1)])
        out.append(oracle.stats(s, d))
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("mode,graphs", [("hash", True), ("hash", False), ("merge", True)])
def test_serving_alone_and_in_the_mix(mode, graphs):
    """Builds replayed from captured graphs (padded batches in fixed slots) or
    launched eagerly give the same results."""
    import torch
    from paper_2510_14050_amd.serve import Server
    ring, n = 6, 40
    wins = small_windows(n)
    want_roll = rolling_want(wins, ring)
    want_win = [oracle.stats(s, d) for s, d in wins]
    # 2^14 link slots: the 18 166 distinct links of these windows pass 60% of
    # them, the at most 5 409 live in the ring stay below half
    kw = dict(mode=mode, link_slots=1 << 14, address_slots=1 << 14, graphs=graphs)
    srv = Server(ring=ring, max_window=1 << 12, max_batch=4, budget_bytes=64 << 20,
                 timing=True, **kw)
    say("serve alone (max_batch 1, serial)", mode)
    alone = Server(ring=ring, max_window=1 << 12, max_batch=1, budget_bytes=64 << 20, **kw)
    rep_alone = alone.run(wins)
    say("serve in the mix (all arrive at once)")
    rep_burst = srv.run(wins)
    say("serve in the mix (Poisson arrivals)")
    arr = synth.poisson_arrivals(9, n, 4000.0)
    rep_poisson = srv.run(wins, arrivals_s=arr)
    torch.cuda.synchronize()
    for rep in (rep_alone, rep_burst, rep_poisson):
        for k, r in enumerate(rep.results):
            assert r.seq == k
            assert r.window_stats.tolist() == want_win[k].tolist(), k
            assert r.rolling_stats.tolist() == want_roll[k].tolist(), k
    # continuous batching really grouped arrivals and overlapped device work
    assert max(rep_burst.batches) > 1
    assert rep_burst.max_in_flight >= 2
    assert rep_burst.device_overlap() >= 1 or max(rep_burst.batches) > 1
    s = rep_poisson.summary()
    assert s["p50_ms"] is not None and s["p99_ms"] >= s["p50_ms"]
    if mode == "hash":  # the small tables forced compactions along the way
        assert rep_burst.compactions >= 1


@pytest.mark.gpu
def test_serving_memory_budget_gates_admission():
    """A budget that only fits the ring plus two micro-batches still serves
    everything correctly (admission waits for memory)."""
    from paper_2510_14050_amd.serve import Server
    ring, n = 4, 30
    wins = small_windows(n, seed=8, lo=10, hi=12)
    want_roll = rolling_want(wins, ring)
    mw = 1 << 12
    budget = 16 * (ring + 2 * 2) * mw + 8 * 2 * mw
    srv = Server(ring=ring, max_window=mw, max_batch=2, budget_bytes=budget,
                 link_slots=1 << 15, address_slots=1 << 14)
    rep = srv.run(wins)
    for k, r in enumerate(rep.results):
        assert r.rolling_stats.tolist() == want_roll[k].tolist(), k
    with pytest.raises(ValueError):
        Server(ring=ring, max_window=mw, max_batch=2, budget_bytes=budget - 1)


@pytest.mark.gpu
@pytest.mark.slow
def test_serving_at_scale_every_arrival():
    """Serving near the full configuration's shape: a ring of 256 windows of
    2^10..2^15 packets (Zipf 1.2 over a pool of 2^20), Poisson arrivals at
    2000 windows/s, hash tables small enough that the rolling state is
    compacted (the 1.98 million distinct links pass 60% of 2^21 link slots;
    at most 0.83 million are live in the ring). Every arrival's window quantities and rolling
    quantities (windows k-255..k by arrival order) equal the oracle's, served
    in the mix and served alone (one window at a time)."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    import torch
    from paper_2510_14050_amd.serve import Server
    ring, n = 256, 800
    wl = synth.Workload("serve_scale_t", 11, 1 << 20, 1.2, 1.2,
                        synth.log_uniform_sizes(11, n, 10, 15))
    wins = [wl.window(w) for w in range(n)]
    say("oracle: every window and every rolling aggregate of", n, "arrivals")
    oracle.stats(wins[0][0][:1], wins[0][1][:1])

    def rolling(k):
        lo = max(0, k - ring + 1)
        return oracle.stats(np.concatenate([wins[j][0] for j in range(lo, k + 1)]),
                            np.concatenate([wins[j][1] for j in range(lo, k + 1)]))
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        roll_jobs = [ex.submit(rolling, k) for k in range(n)]
        want_win = list(ex.map(lambda w: oracle.stats(*w), wins))
        want_roll = [j.result() for j in roll_jobs]
    kw = dict(ring=ring, max_window=1 << 15, budget_bytes=256 << 20,
              link_slots=1 << 21, address_slots=1 << 22)
    arr = synth.poisson_arrivals(12, n, 2000.0)
    say("serve in the mix (Poisson arrivals, micro-batches of up to 16)")
    rep_mix = Server(max_batch=16, **kw).run(wins, arrivals_s=arr - arr[0])
    say("serve alone (one window at a time)")
    rep_alone = Server(max_batch=1, **kw).run(wins)
    torch.cuda.synchronize()
    for rep in (rep_mix, rep_alone):
        for k, r in enumerate(rep.results):
            assert r.seq == k
            assert r.window_stats.tolist() == want_win[k].tolist(), k
            assert r.rolling_stats.tolist() == want_roll[k].tolist(), k
        assert rep.compactions >= 1, rep.compactions
    s = rep_mix.summary()
    say("in the mix:", {k: s[k] for k in ("p50_ms", "p99_ms", "mean_batch", "max_in_flight")},
        "compactions", rep_mix.compactions)
