"""Parity of the HIP path (through the C ABI) with the CPU oracle.

All arithmetic is integer, so the bar is bit-exact equality of every output:
the sorted COO arrays (keys, counts, nnz) and the eight quantities.
Sizes span several tiles with ragged tails, empty inputs, single packets,
long runs that cross many tiles, and the full workload sizes.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2510_14050_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_2510_14050_amd import ns
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm GPU"
    ns.load()
    return torch, ns


def up32(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).cuda()


def zipf_packets(seed, n, pool=4096, s=1.2):
    wl = synth.Workload("t", seed, pool, s, s + 0.1, np.array([n], np.int64))
    return wl.window(0)


def build_and_check(torch, ns, src, dst, ws=None):
    n = src.size
    ws = ws or ns.Workspace(n, 1)
    m = ns.Matrix(n)
    ns.build_matrix(up32(torch, src), up32(torch, dst), m, ws)
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    ns.stats(m, out, ws)
    torch.cuda.synchronize()
    k, c = m.numpy()
    ok, oc = oracle.build_matrix(src, dst)
    assert m.packets == n
    assert k.size == ok.size, (k.size, ok.size)
    assert np.array_equal(k, ok)
    assert np.array_equal(c, oc)
    want = oracle.stats(src, dst)
    assert ns.stats_numpy(out).tolist() == want.tolist()
    return m


SIZES = [0, 1, 2, 7, 255, 256, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097,
         8191, 8193, 12345, 16383, 16384, 16385, 65537, 131072]


@pytest.mark.parametrize("n", SIZES)
def test_build_and_stats_sizes(gpu, n):
    torch, ns = gpu
    say("build_and_stats n=", n)
    src, dst = zipf_packets(100 + n, n, pool=max(4, n // 8))
    build_and_check(torch, ns, src, dst)


def patterns():
    rng = np.random.default_rng(7)
    n = 100_000
    yield "identical", np.full(n, 0xC0A80001, np.uint32), np.full(n, 0x0A000001, np.uint32)
    yield "all_distinct", rng.permutation(1 << 20)[:n].astype(np.uint32) * 4093, \
        rng.permutation(1 << 20)[:n].astype(np.uint32) * 17
    t = (rng.permutation(1 << 20)[:70_000].astype(np.uint32) << 8) | 3
    yield "scanner", np.full(t.size, 0xFFFFFFFF, np.uint32), t
    yield "sink", t, np.zeros(t.size, np.uint32)
    s, d = zipf_packets(5, 50_000, pool=64)
    yield "sign_flip", s ^ np.uint32(0x80000000), d ^ np.uint32(0x80000000)
    ext = np.array([0, 0xFFFFFFFF, 0x7FFFFFFF, 0x80000000], np.uint32)
    yield "extremes", ext[rng.integers(0, 4, 30_000)], ext[rng.integers(0, 4, 30_000)]
    S = rng.integers(0, 2**32, 37, dtype=np.uint64).astype(np.uint32)
    D = rng.integers(0, 2**32, 53, dtype=np.uint64).astype(np.uint32)
    yield "grid", np.repeat(np.repeat(S, 53), 3), np.repeat(np.tile(D, 37), 3)
    # one hot link in the middle of otherwise distinct traffic: a run across tiles
    a = np.arange(60_000, dtype=np.uint32)
    a[20_000:45_000] = 12345
    yield "hot_link", a, a


@pytest.mark.parametrize("name,src,dst", list(patterns()), ids=[p[0] for p in patterns()])
def test_patterns(gpu, name, src, dst):
    torch, ns = gpu
    say("pattern", name)
    build_and_check(torch, ns, src, dst)


def run_batch(torch, ns, src, dst, sizes, graph=True, agg=True, win=True, tune=None, ws=None,
              windows=True):
    off = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    N, W = int(off[-1]), len(sizes)
    ws = ws or ns.Workspace(N, W)
    out = torch.full((W, 8), -1, dtype=torch.int64, device="cuda") if windows else None
    m = ns.Matrix(N) if agg else None
    ms = torch.full((8,), -1, dtype=torch.int64, device="cuda") if agg else None
    wm = ns.BatchMatrices(N, W) if win else None
    ns.batch_stats(up32(torch, src), up32(torch, dst), torch.from_numpy(off).cuda(), out, ws,
                   agg=m, agg_stats=ms, win=wm, tune=tune, graph=graph)
    torch.cuda.synchronize()
    return off, out, m, ms, wm


def check_batch(ns, src, dst, off, out, m, ms, wm):
    if out is not None:
        want = oracle.stats_windows(src, dst, off.astype(np.uint64))
        got = ns.stats_numpy(out)
        bad = np.nonzero((got != want).any(axis=1))[0]
        assert bad.size == 0, f"windows {bad[:5]}: got {got[bad[:2]]} want {want[bad[:2]]}"
    if m is not None:
        k, c = m.numpy()
        ok, oc = oracle.build_matrix(src, dst)
        assert np.array_equal(k, ok) and np.array_equal(c, oc)
        assert m.packets == src.size
        assert ns.stats_numpy(ms).tolist() == oracle.stats(src, dst).tolist()
    if wm is not None:
        nz = wm.nnz.cpu().numpy()
        keys = wm.keys.cpu().numpy().view(np.uint64)
        cnts = wm.counts.cpu().numpy().view(np.uint64)
        for w in range(len(off) - 1):
            a, b = int(off[w]), int(off[w + 1])
            ok, oc = oracle.build_matrix(src[a:b], dst[a:b])
            assert nz[w] == ok.size, w
            assert np.array_equal(keys[a:a + ok.size], ok), w
            assert np.array_equal(cnts[a:a + ok.size], oc), w


RAGGED = [0, 5, 3000, 0, 70_000, 1, 4096, 4097, 0, 2048, 2049, 131072, 17, 0]


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
def test_batch_ragged(gpu, graph):
    torch, ns = gpu
    say("batch ragged graph=", graph)
    N = sum(RAGGED)
    src, dst = zipf_packets(77, N, pool=2000)
    res = run_batch(torch, ns, src, dst, RAGGED, graph=graph)
    check_batch(ns, src, dst, *res)


def test_batch_all_empty_and_single(gpu):
    torch, ns = gpu
    say("batch all empty")
    e = np.zeros(0, np.uint32)
    res = run_batch(torch, ns, e, e, [0, 0, 0])
    check_batch(ns, e, e, *res)
    say("batch single window of one packet")
    one = np.array([0xFFFFFFFF], np.uint32)
    res = run_batch(torch, ns, one, one ^ np.uint32(1), [1])
    check_batch(ns, one, one ^ np.uint32(1), *res)


@pytest.mark.parametrize("shape", [(256, 8, 4), (256, 16, 8), (512, 8, 8), (512, 16, 4),
                                   (512, 16, 16)])
def test_batch_tuning_shapes(gpu, shape):
    """Radix tiles and run tiles on ragged windows with their aggregate and
    window matrices."""
    torch, ns = gpu
    say("batch tuning", shape)
    sizes = [9000, 1, 0, 40000, 33333, 2 * 8192 + 3]
    src, dst = zipf_packets(91, sum(sizes), pool=3000)
    t = ns.tuning(sort_block=shape[0], sort_items=shape[1], digit_bits=8, scan_items=shape[2])
    res = run_batch(torch, ns, src, dst, sizes, tune=t)
    check_batch(ns, src, dst, *res)


@pytest.mark.parametrize("scan", [4, 8, 16])
@pytest.mark.parametrize("n", [8191, 8192, 8193, 65536 * 3 + 5, 1_000_003])
def test_run_length_tiles_single_segment(gpu, n, scan):
    """The run-length pass on one long segment (the aggregate alone) for each
    run tile, around the tile sizes; long runs of equal keys cross tile ends
    (a pool of 40 addresses)."""
    torch, ns = gpu
    say("run-length tiles", n, scan)
    src, dst = zipf_packets(700 + n % 13, n, pool=40)
    t = ns.tuning(scan_items=scan)
    res = run_batch(torch, ns, src, dst, [n], tune=t, win=False, windows=False)
    check_batch(ns, src, dst, *res)


@pytest.mark.parametrize("shape", [(256, 16), (512, 8)])
def test_batch_layered_tickets(gpu, shape):
    """Few windows of similar length take radix tickets layer by layer; some
    windows have one tile fewer (their tickets in the last layer are skipped)
    and one is empty."""
    torch, ns = gpu
    rng = np.random.default_rng(3)
    tile = shape[0] * shape[1]
    sizes = [int(x) for x in rng.integers(4 * tile + 1, 5 * tile, 31)] + [0, 4 * tile - 7]
    say("layered tickets", shape, len(sizes), "windows")
    src, dst = zipf_packets(44, sum(sizes), pool=5000)
    t = ns.tuning(sort_block=shape[0], sort_items=shape[1])
    for graph in (True, False):
        res = run_batch(torch, ns, src, dst, sizes, tune=t, graph=graph)
        check_batch(ns, src, dst, *res)


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
@pytest.mark.parametrize("W", [2, 3, 5, 64, 127, 128, 129, 200])
def test_batch_aggregate_window_counts(gpu, W, graph):
    """The aggregate and every window over a range of window counts (odd,
    powers of two, either side of 128), with and without the per-window
    matrices requested, with an empty window mixed in."""
    torch, ns = gpu
    rng = np.random.default_rng(W)
    sizes = [int(x) for x in rng.integers(0, 3000, W)]
    sizes[W // 2] = 0
    say("aggregate, windows:", W, "graph" if graph else "eager")
    src, dst = zipf_packets(500 + W, sum(sizes), pool=700)
    for win in (True, False):
        res = run_batch(torch, ns, src, dst, sizes, graph=graph, win=win)
        check_batch(ns, src, dst, *res)


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
@pytest.mark.parametrize("case", ["one", "two", "ragged", "w129", "all_empty", "chunked"])
def test_batch_aggregate_alone(gpu, case, graph):
    """ns_batch_stats with the aggregate as its only output (no per-window
    quantities): the aggregate's matrix and quantities against the oracle,
    for one window, several, ragged and empty ones, and the chunked passes."""
    torch, ns = gpu
    rng = np.random.default_rng(77)
    sizes = {"one": [70_001], "two": [4097, 12_345], "ragged": RAGGED,
             "w129": [int(x) for x in rng.integers(0, 2000, 129)], "all_empty": [0, 0, 0],
             "chunked": [100_000, 0, 33_333]}[case]
    t = ns.tuning(chunked_min=1) if case == "chunked" else None
    say("aggregate alone", case, "graph" if graph else "eager")
    src, dst = zipf_packets(900 + len(sizes), sum(sizes), pool=1500)
    res = run_batch(torch, ns, src, dst, sizes, graph=graph, win=False, windows=False, tune=t)
    check_batch(ns, src, dst, *res)


CHUNKED_CASES = {
    "ragged_agg": RAGGED,
    "one_window": [300_001],
    "one_empty": [0],
    "one_packet": [1],
    "one_tile_plus": [4097],
}


@pytest.mark.parametrize("bits", [8, 11])
@pytest.mark.parametrize("shape", [(256, 8), (256, 16), (512, 8), (512, 16)])
@pytest.mark.parametrize("case", list(CHUNKED_CASES))
def test_batch_chunked_single_segment(gpu, case, shape, bits):
    """Single segments (the aggregate, or a batch of one window) forced onto
    the chunked passes, with byte digits and with 11-bit digits (6 key passes,
    3 column passes): same results as the oracle."""
    torch, ns = gpu
    sizes = CHUNKED_CASES[case]
    say("chunked single segment", case, shape, "digit bits", bits)
    src, dst = zipf_packets(31 + len(sizes), sum(sizes), pool=2500)
    t = ns.tuning(sort_block=shape[0], sort_items=shape[1], chunked_min=1, digit_bits=bits)
    for graph in (True, False):
        res = run_batch(torch, ns, src, dst, sizes, tune=t, graph=graph)
        check_batch(ns, src, dst, *res)


@pytest.mark.parametrize("bits", [8, 11])
@pytest.mark.parametrize("name", ["hot_link", "extremes", "scanner", "identical"])
def test_batch_chunked_patterns(gpu, name, bits):
    torch, ns = gpu
    src, dst = {p[0]: p[1:] for p in patterns()}[name]
    say("chunked pattern", name, "digit bits", bits)
    t = ns.tuning(chunked_min=1, digit_bits=bits)
    res = run_batch(torch, ns, src, dst, [src.size], tune=t)
    check_batch(ns, src, dst, *res)


@pytest.mark.parametrize("n", [2047, 2048, 2049, 8191, 8193, 32767, 32769, 100_003])
def test_wide_digits_tile_and_chunk_edges(gpu, n):
    """11-bit digits around the digit count (2048), the tile (8192 keys) and
    the chunk (4 tiles): one segment on the chunked passes, through the
    aggregate-only call, against the oracle."""
    torch, ns = gpu
    say("wide digits, n =", n)
    src, dst = zipf_packets(4000 + n % 97, n, pool=3000, s=1.1)
    t = ns.tuning(chunked_min=1, digit_bits=11)
    res = run_batch(torch, ns, src, dst, [n], tune=t, win=False, windows=False)
    check_batch(ns, src, dst, *res)


def test_single_window_above_chunked_threshold(gpu):
    """A window of 2^24 + 12345 packets takes the chunked passes by default
    (build_matrix and the statistics of its matrix)."""
    torch, ns = gpu
    n = (1 << 24) + 12345
    say("single window, chunked by default, n=", n)
    src, dst = zipf_packets(2024, n, pool=1 << 18, s=1.1)
    build_and_check(torch, ns, src, dst)


def test_graph_replays_match_eager(gpu):
    """A cached graph replayed on new data in the same buffers, with eager
    work and synchronisation between replays, matches the oracle each time."""
    torch, ns = gpu
    sizes = [5000, 0, 20000, 777, 60000]
    N, W = sum(sizes), len(sizes)
    off = np.zeros(W + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    ws = ns.Workspace(N, W)
    s_t = torch.empty(N, dtype=torch.int32, device="cuda")
    d_t = torch.empty(N, dtype=torch.int32, device="cuda")
    o_t = torch.from_numpy(off).cuda()
    out = torch.zeros((W, 8), dtype=torch.int64, device="cuda")
    m = ns.Matrix(N)
    ms = torch.zeros(8, dtype=torch.int64, device="cuda")
    for rep in range(4):
        say("graph replay", rep)
        src, dst = zipf_packets(300 + rep, N, pool=500 + 300 * rep)
        s_t.copy_(up32(torch, src))
        d_t.copy_(up32(torch, dst))
        ns.batch_stats(s_t, d_t, o_t, out, ws, agg=m, agg_stats=ms)
        torch.cuda.synchronize()
        check_batch(ns, src, dst, off, out, m, ms, None)
        # unrelated eager work on the same stream between replays
        tmp = ns.Matrix(1000)
        ns.build_matrix(s_t[:1000], d_t[:1000], tmp, ws)
        torch.cuda.synchronize()


def test_accumulate_add_subtract(gpu):
    torch, ns = gpu
    say("accumulate")
    s1, d1 = zipf_packets(11, 50_000, pool=800)
    s2, d2 = zipf_packets(12, 30_000, pool=800)
    ws = ns.Workspace(200_000, 1)
    A, B = ns.Matrix(50_000), ns.Matrix(30_000)
    ns.build_matrix(up32(torch, s1), up32(torch, d1), A, ws)
    ns.build_matrix(up32(torch, s2), up32(torch, d2), B, ws)
    C = ns.Matrix(80_000)
    ns.accumulate(A, B, 1, C, ws)
    D = ns.Matrix(80_000)
    ns.accumulate(C, B, -1, D, ws)
    E = ns.Matrix(80_000)
    ns.accumulate(B, A, 1, E, ws)
    torch.cuda.synchronize()
    assert ns.device_status() == 0
    ka, ca = oracle.build_matrix(s1, d1)
    kb, cb = oracle.build_matrix(s2, d2)
    kc, cc = oracle.accumulate(ka, ca, kb, cb, 1)
    for M, (wk, wc) in [(C, (kc, cc)), (D, (ka, ca)), (E, (kc, cc))]:
        k, c = M.numpy()
        assert np.array_equal(k, wk) and np.array_equal(c, wc)
    assert C.packets == 80_000 and D.packets == 50_000
    # stats of the sum = stats of the concatenated packets
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    ns.stats(C, out, ws)
    torch.cuda.synchronize()
    want = oracle.stats(np.concatenate([s1, s2]), np.concatenate([d1, d2]))
    assert ns.stats_numpy(out).tolist() == want.tolist()
    # subtracting everything leaves the empty matrix
    Z = ns.Matrix(50_000)
    ns.accumulate(A, A, -1, Z, ws)
    torch.cuda.synchronize()
    assert Z.nnz() == 0 and Z.packets == 0
    ns.stats(Z, out, ws)
    torch.cuda.synchronize()
    assert ns.stats_numpy(out).tolist() == [0] * 8


def test_accumulate_with_its_own_small_workspace(gpu):
    """ns_accumulate with a workspace of exactly ns_accumulate_workspace_size
    bytes (one ticket and the merge tiles' look-back words): a sum and a
    difference in a row on the one workspace, against the oracle."""
    torch, ns = gpu
    say("accumulate, merge workspace")
    s1, d1 = zipf_packets(21, 70_000, pool=900)
    s2, d2 = zipf_packets(22, 45_000, pool=900)
    ws = ns.Workspace(70_000, 1)
    A, B = ns.Matrix(70_000), ns.Matrix(45_000)
    ns.build_matrix(up32(torch, s1), up32(torch, d1), A, ws)
    ns.build_matrix(up32(torch, s2), up32(torch, d2), B, ws)
    mw = ns.MergeWorkspace(115_000, 45_000)  # the larger of the two calls' bounds
    assert mw.nbytes < 4096 < ws.nbytes
    C, D = ns.Matrix(115_000), ns.Matrix(115_000)
    ns.accumulate(A, B, 1, C, mw)
    ns.accumulate(C, B, -1, D, mw)
    torch.cuda.synchronize()
    assert ns.device_status() == 0
    ka, ca = oracle.build_matrix(s1, d1)
    kb, cb = oracle.build_matrix(s2, d2)
    kc, cc = oracle.accumulate(ka, ca, kb, cb, 1)
    for M, (wk, wc) in [(C, (kc, cc)), (D, (ka, ca))]:
        k, c = M.numpy()
        assert np.array_equal(k, wk) and np.array_equal(c, wc)
    assert C.packets == 115_000 and D.packets == 70_000


def test_accumulate_edge_cases(gpu):
    torch, ns = gpu
    say("accumulate edges")
    ws = ns.Workspace(10_000, 1)
    empty = ns.Matrix(0)
    ns.build_matrix(torch.empty(0, dtype=torch.int32, device="cuda"),
                    torch.empty(0, dtype=torch.int32, device="cuda"), empty, ws)
    s, d = zipf_packets(3, 5000, pool=50)
    A = ns.Matrix(5000)
    ns.build_matrix(up32(torch, s), up32(torch, d), A, ws)
    out1, out2, out3 = ns.Matrix(5000), ns.Matrix(5000), ns.Matrix(1)
    ns.accumulate(A, empty, 1, out1, ws)
    ns.accumulate(empty, A, 1, out2, ws)
    ns.accumulate(empty, empty, 1, out3, ws)
    torch.cuda.synchronize()
    ka, ca = oracle.build_matrix(s, d)
    for M in (out1, out2):
        k, c = M.numpy()
        assert np.array_equal(k, ka) and np.array_equal(c, ca)
    assert out3.nnz() == 0
    # device-detected underflow: B has an entry A lacks (same packet totals)
    s2 = s.copy()
    s2[0] = 0xDEADBEEF
    B = ns.Matrix(5000)
    ns.build_matrix(up32(torch, s2), up32(torch, d), B, ws)
    bad = ns.Matrix(5000)
    ns.accumulate(A, B, -1, bad, ws)
    assert ns.device_status() == -5
    assert ns.device_status() == 0  # reading clears the word


@pytest.mark.parametrize("key", ["one_window", "windows64"])
def test_workload_full_size(gpu, key):
    """The one-window and the 64-window workloads at their full sizes, in the
    launch configuration the benchmark times (graph, aggregate + its stats)."""
    torch, ns = gpu
    say("workload", key)
    wl = synth.WORKLOADS[key]()
    src, dst = wl.concat()
    res = run_batch(torch, ns, src, dst, list(wl.sizes), win=False)
    check_batch(ns, src, dst, *res)


def test_workload_uneven1024(gpu):
    torch, ns = gpu
    say("workload uneven1024")
    wl = synth.uneven1024()
    src, dst = wl.concat()
    res = run_batch(torch, ns, src, dst, list(wl.sizes), agg=False, win=False)
    check_batch(ns, src, dst, *res)


@pytest.mark.parametrize("bits", [8, 11])
def test_workload_uneven1024_with_aggregate(gpu, bits):
    """1024 uneven windows with their aggregate: the aggregate's 3.5 x 10^7 keys
    take the chunked passes with more chunks than chunk-scan blocks (several
    chunk rows per block), with byte and with 11-bit digits; matrix and
    statistics against the oracle."""
    torch, ns = gpu
    say("workload uneven1024 + aggregate, digit bits", bits)
    wl = synth.uneven1024()
    src, dst = wl.concat()
    assert src.size >= (1 << 24) and src.size > 1024 * 4 * 8192  # chunked, > 1024 chunks
    res = run_batch(torch, ns, src, dst, list(wl.sizes), agg=True, win=False,
                    tune=ns.tuning(digit_bits=bits, chunked_min=1 << 24))
    check_batch(ns, src, dst, *res)


# Batches of at most 8192 packets in total run each window's whole pipeline in
# one workgroup's LDS (k_small); one more packet takes the multi-kernel path.
SMALL_BATCHES = {
    "one_8192": [8192],
    "one_8191": [8191],
    "one_1": [1],
    "empty_and_small": [0, 1, 0, 2, 17, 0],
    "two_to_8192": [4096, 4096],
    "sixteen": [512] * 15 + [512],
    "four_2000": [2000] * 4,
    "ragged_8192": [3000, 1, 0, 2048, 2049, 1000, 94],
    "ragged_8193": [3000, 1, 0, 2048, 2049, 1000, 95],
    "many_empty": [0] * 300 + [8000] + [0] * 200,
}


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("name", sorted(SMALL_BATCHES))
def test_small_batch_path(gpu, name, graph):
    """Every window's quantities and matrix against the oracle, with and
    without the aggregate, at and beyond the one-workgroup threshold."""
    torch, ns = gpu
    sizes = SMALL_BATCHES[name]
    say("small batch", name, "graph" if graph else "eager")
    src, dst = zipf_packets(300 + len(sizes), sum(sizes), pool=700)
    for agg in (False, True):
        res = run_batch(torch, ns, src, dst, sizes, graph=graph, agg=agg)
        assert ns.device_status() == 0
        check_batch(ns, src, dst, *res)


@pytest.mark.parametrize("n", [8192, 8193])
@pytest.mark.parametrize("pattern", ["identical", "fan_out", "fan_in", "distinct", "two_rows",
                                     "blocks", "all_ones"])
def test_small_batch_extremes(gpu, pattern, n):
    """Windows of 8192 packets whose counts, fan-out or fan-in reach 8192 (the
    largest values the one-workgroup path packs into 16 bits), runs that span
    a few threads' positions, and the all-ones key; the same patterns one
    packet over, on the multi-kernel path."""
    torch, ns = gpu
    i = np.arange(n, dtype=np.uint32)
    if pattern == "identical":
        src, dst = np.full(n, 7, np.uint32), np.full(n, 0xFFFFFFFF, np.uint32)
    elif pattern == "fan_out":
        src, dst = np.full(n, 0x80000000, np.uint32), (i * 2654435761).astype(np.uint32)
    elif pattern == "fan_in":
        src, dst = (i * 2654435761 + 1).astype(np.uint32), np.zeros(n, np.uint32)
    elif pattern == "distinct":
        src, dst = (i * 40503).astype(np.uint32), (i * 2654435761).astype(np.uint32)
    elif pattern == "two_rows":
        src, dst = (i & 1).astype(np.uint32), (i >> 1).astype(np.uint32)
    elif pattern == "blocks":
        src, dst = (i // 37).astype(np.uint32), ((i // 1000) * 77).astype(np.uint32)
    else:  # a third of the packets on the all-ones key, the rest spread below it
        src = np.where(i % 3 == 0, 0xFFFFFFFF, i * 2654435761).astype(np.uint32)
        dst = np.where(i % 3 == 0, 0xFFFFFFFF, i // 5).astype(np.uint32)
    say("small batch extremes", pattern)
    res = run_batch(torch, ns, src, dst, [n], graph=False, agg=False)
    assert ns.device_status() == 0
    check_batch(ns, src, dst, *res)
