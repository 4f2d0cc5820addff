"""Matrices holding 2^32 packets or more: the eight quantities of a matrix
whose link counts and row / column sums need 64 bits (the aggregate of an
out-of-core build over more packets than 32-bit sums can hold, Sec. III-C),
against the oracle and against closed forms."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def device_matrix(torch, ns, keys, counts):
    k = torch.from_numpy(keys.view(np.int64)).cuda()
    c = torch.from_numpy(counts.view(np.int64)).cuda()
    nnz = torch.tensor([keys.size], dtype=torch.int64, device="cuda")
    return ns.Matrix.wrap(k, c, nnz, keys.size, int(counts.sum(dtype=np.uint64)))


@pytest.mark.parametrize("n,rows,cols,seed", [(1, 1, 1, 1), (700, 30, 40, 2), (5000, 300, 300, 3),
                                              (200_003, 5000, 9000, 4)])
def test_stats_with_counts_past_2p32(n, rows, cols, seed):
    """Random sorted matrices with counts up to 2^40 (so every run sum and
    tile sum passes 2^32) against the oracle's quantities of the same matrix."""
    import torch
    from paper_2510_14050_amd import ns
    say("wide counts", n, rows, cols)
    rng = np.random.default_rng(seed)
    src = rng.integers(0, rows, 3 * n).astype(np.uint64) * np.uint64(0x01000193) + np.uint64(7)
    dst = rng.integers(0, cols, 3 * n).astype(np.uint64) * np.uint64(0x9E3779B1) % np.uint64(1 << 32)
    keys = np.unique((src << np.uint64(32)) | dst)[:n]
    counts = rng.integers(1, 1 << 40, keys.size, dtype=np.uint64)
    counts[::7] = rng.integers(1, 4, counts[::7].size, dtype=np.uint64)  # small ones mixed in
    m = device_matrix(torch, ns, keys, counts)
    assert m.packets > (1 << 32) or keys.size == 1
    if keys.size == 1:  # one link of more than 2^32 packets
        counts[0] = np.uint64((1 << 33) + 5)
        m = device_matrix(torch, ns, keys, counts)
    ws = ns.Workspace(keys.size, 1)
    out = torch.full((8,), -1, dtype=torch.int64, device="cuda")
    ns.stats(m, out, ws)
    torch.cuda.synchronize()
    assert ns.device_status() == 0
    want = oracle.stats_matrix(keys, counts)
    assert ns.stats_numpy(out).tolist() == want.tolist()
    assert int(want[0]) == int(counts.sum(dtype=np.uint64))


@pytest.mark.slow
def test_streamed_build_past_2p32_packets():
    """2^32 + 2^20 + 5 packets streamed from page-locked host memory through
    ns_build_matrix_streamed in sub-partitions of 2^27 (a small device
    footprint), then ns_stats of the aggregate: one link (A, B) repeated
    2^32 + 5 times and a grid of 2^10 sources x 2^10 destinations once each,
    spread over the whole input. The aggregate's entries and its eight
    quantities follow in closed form."""
    import torch
    from paper_2510_14050_amd import ns
    torch.cuda.empty_cache()
    hot = (1 << 32) + 5
    g = 1 << 20
    n = hot + g
    A, B = 0xC0A80001, 0x08080808
    say("filling", n, "packets in page-locked host memory")
    s_t = torch.empty(n, dtype=torch.int32, pin_memory=True)
    d_t = torch.empty(n, dtype=torch.int32, pin_memory=True)
    src, dst = s_t.numpy().view(np.uint32), d_t.numpy().view(np.uint32)
    src.fill(A)
    dst.fill(B)
    k = np.arange(g, dtype=np.int64)
    pos = k * 4096 + 7
    src[pos] = (0x0A000000 + (k >> 10)).astype(np.uint32)
    dst[pos] = (0x0B000000 + (k & 1023)).astype(np.uint32)
    del k, pos
    batch = 1 << 27
    out = ns.Matrix(g + 1 + batch)
    sws = ns.StreamWorkspace(batch, out.capacity)
    say("ns_build_matrix_streamed:", (n + batch - 1) // batch, "sub-partitions")
    ns.build_matrix_streamed(s_t, d_t, out, sws)
    torch.cuda.synchronize()
    assert ns.device_status() == 0
    assert out.packets == n and out.nnz() == g + 1
    del sws
    # the aggregate's entries are bounded by its links (g + 1), not its capacity
    agg = ns.Matrix.wrap(out.keys, out.counts, out.nnz_t, g + 1, out.packets)
    ws = ns.Workspace(g + 1, 1)
    st = torch.full((8,), -1, dtype=torch.int64, device="cuda")
    say("ns_stats of the aggregate")
    ns.stats(agg, st, ws)
    torch.cuda.synchronize()
    assert ns.device_status() == 0
    got = [int(x) for x in ns.stats_numpy(st)]
    assert got == [n, g + 1, 1024 + 1, 1024 + 1, hot, 1024, hot, 1024], got
    keys, counts = out.numpy()
    ks = np.arange(g, dtype=np.uint64)
    grid = ((np.uint64(0x0A000000) + (ks >> np.uint64(10))) << np.uint64(32)) | \
        (np.uint64(0x0B000000) + (ks & np.uint64(1023)))
    want_k = np.sort(np.append(grid, np.uint64((A << 32) | B)))
    assert np.array_equal(keys, want_k)
    want_c = np.where(want_k == np.uint64((A << 32) | B), np.uint64(hot), np.uint64(1))
    assert np.array_equal(counts, want_c)
    del out, ws
    torch.cuda.empty_cache()
