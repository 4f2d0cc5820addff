"""Full-size check of the 2^30-packet aggregate (8192 windows of 2^17 with a
scanner and a sink), in the benchmark's launch configuration.

The oracle cannot sort 2^30 keys within a test's time, so parity here is:
* properties that hold at any size (sorted strictly increasing keys, counts
  >= 1 summing to 2^30, valid packets = 2^30, the invariants between the eight
  quantities, the scanner's 2^16 distinct targets),
* the eight quantities recomputed by the oracle from the GPU's own matrix
  (checks the statistics pass at full size),
* sampled rows of the matrix recomputed by the oracle from the packets of the
  sampled sources (checks the matrix construction at full size).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2510_14050_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def test_aggregate_2p30_full_size():
    import torch
    from paper_2510_14050_amd import ns
    dev = torch.device("cuda:0")
    wl = synth.aggregate_2p30()
    N = wl.total_packets
    assert N == 1 << 30
    say("generating 2^30 packets on the device")
    src_t, dst_t = wl.device_concat(dev)
    W = wl.num_windows
    off = torch.from_numpy(wl.offsets).to(dev)
    ws = ns.Workspace(N, W, device=dev)
    agg = ns.Matrix(N, device=dev)
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    win_st = torch.zeros((W, 8), dtype=torch.int64, device=dev)
    say("ns_batch_stats: 8192 windows + aggregate")
    ns.batch_stats(src_t, dst_t, off, win_st, ws, agg=agg, agg_stats=st)
    torch.cuda.synchronize()
    got = ns.stats_numpy(st).copy()
    per_win = ns.stats_numpy(win_st).copy()
    v, links, ns_, nd, msp, mfo, mdp, mfi = [int(x) for x in got]
    say("stats", got.tolist())
    assert v == N
    assert links <= v and links >= max(mfo, mfi)
    assert max(ns_, nd) <= links
    assert mfo <= min(nd, msp) and mfi <= min(ns_, mdp)
    assert mfo >= 1 << 16 and mfi >= 1 << 16   # scanner / sink reach 2^16 peers
    say("copying the matrix to the host")
    keys, counts = agg.numpy()
    assert keys.size == links
    assert np.all(keys[1:] > keys[:-1])
    assert counts.min() >= 1 and int(counts.sum()) == N
    say("oracle statistics of the GPU matrix")
    assert oracle.stats_matrix(keys, counts).tolist() == got.tolist()
    say("sampled windows against the oracle")
    src = synth.as_u32(src_t)
    dst = synth.as_u32(dst_t)
    del src_t, dst_t
    o = wl.offsets
    for w in [0, 1, 4095, 8191] + list(np.random.default_rng(1).integers(0, W, 8)):
        a, b = int(o[w]), int(o[w + 1])
        assert per_win[w].tolist() == oracle.stats(src[a:b], dst[a:b]).tolist(), w
    assert int(per_win[:, 0].sum()) == N
    say("sampled rows against the oracle")
    rng = np.random.default_rng(0)
    rows = keys >> np.uint64(32)
    sample = np.unique(np.concatenate([
        np.array([wl.scanner, int(wl.sources[0]), int(wl.sources[-1])], np.uint64),
        rows[rng.integers(0, rows.size, 40)],
        rows[:1], rows[-1:]])).astype(np.uint32)
    pos = np.minimum(np.searchsorted(sample, src), sample.size - 1)
    mask = sample[pos] == src
    ok, oc = oracle.build_matrix(src[mask], dst[mask])
    sel = np.isin(rows.astype(np.uint32), sample)
    assert np.array_equal(keys[sel], ok)
    assert np.array_equal(counts[sel], oc)
    # the scanner row: exactly 2^16 distinct targets, 1% of every window's packets
    srow = keys[rows == np.uint64(wl.scanner)]
    assert srow.size == 1 << 16
    assert int(counts[rows == np.uint64(wl.scanner)].sum()) == 8192 * wl.scan_count(1 << 17)
