"""Statistics of a matrix given in hypersparse CSR form (the challenge's
matrix files, Sec. IV "Data Representation"): the eight quantities must equal
the oracle's for the same matrix, bit for bit."""
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


def to_csr(keys, counts, empty_rows=()):
    """Hypersparse CSR arrays of a sorted COO matrix; `empty_rows` are extra
    stored rows without entries (source addresses absent from the matrix)."""
    src = (keys >> np.uint64(32)).astype(np.uint32)
    cols = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    rows, starts = np.unique(src, return_index=True)
    row_ptr = np.append(starts, keys.size).astype(np.uint64)
    if len(empty_rows):
        extra = np.setdiff1d(np.asarray(empty_rows, np.uint32), rows)
        all_rows = np.union1d(rows, extra)
        ptr = np.searchsorted(src, all_rows, side="left").astype(np.uint64)
        rows, row_ptr = all_rows, np.append(ptr, keys.size).astype(np.uint64)
    return rows, row_ptr, cols, counts.astype(np.uint64)


def run_csr(torch, ns, rows, row_ptr, cols, vals, packets):
    dev = "cuda"
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).to(dev)
    out = torch.full((8,), -1, dtype=torch.int64, device=dev)
    ns.stats_csr(t(rows.astype(np.uint32), np.int32), t(row_ptr.astype(np.uint64), np.int64),
                 t(cols.astype(np.uint32), np.int32), t(vals.astype(np.uint64), np.int64),
                 packets, out)
    torch.cuda.synchronize()
    return ns.stats_numpy(out).tolist()


def packets(seed, n, pool, s=1.2):
    wl = synth.Workload("t", seed, pool, s, s + 0.1, np.array([n], np.int64))
    return wl.window(0)


@pytest.mark.parametrize("n,pool", [(1, 1), (7, 2), (5000, 40), (200_003, 3000), (131_072, 1 << 16)])
def test_csr_stats_match_oracle(gpu, n, pool):
    torch, ns = gpu
    say("csr", n, pool)
    src, dst = packets(31, n, pool)
    k, c = oracle.build_matrix(src, dst)
    got = run_csr(torch, ns, *to_csr(k, c), n)
    assert ns.device_status() == 0
    assert got == oracle.stats(src, dst).tolist()


def test_csr_empty_matrix_and_empty_rows(gpu):
    torch, ns = gpu
    say("csr empty")
    z = np.zeros(0, np.uint64)
    got = run_csr(torch, ns, np.zeros(0, np.uint32), np.zeros(1, np.uint64),
                  np.zeros(0, np.uint32), z, 0)
    assert got == [0] * 8
    src, dst = packets(32, 20_000, 500)
    k, c = oracle.build_matrix(src, dst)
    rows, row_ptr, cols, vals = to_csr(k, c, empty_rows=[0, 7, 0xFFFFFFFF, 123456789])
    got = run_csr(torch, ns, rows, row_ptr, cols, vals, src.size)
    assert ns.device_status() == 0
    assert got == oracle.stats(src, dst).tolist()


def test_csr_scanner_and_hot_row(gpu):
    """One source to 2^16 destinations once each, plus a hot link."""
    torch, ns = gpu
    say("csr scanner")
    m = 1 << 16
    src = np.concatenate([np.full(m, 0xABCDEF01, np.uint32), np.full(5000, 3, np.uint32)])
    dst = np.concatenate([np.arange(m, dtype=np.uint32) * 7, np.full(5000, 9, np.uint32)])
    k, c = oracle.build_matrix(src, dst)
    got = run_csr(torch, ns, *to_csr(k, c), src.size)
    assert got == oracle.stats(src, dst).tolist()
    assert got[5] == m  # fan-out of the scanner


def test_csr_aggregate_of_the_64_window_workload(gpu):
    """The 64-window workload's aggregate (8.4 x 10^6 packets) as CSR."""
    torch, ns = gpu
    say("csr windows64 aggregate")
    src, dst = synth.WORKLOADS["windows64"]().concat()
    k, c = oracle.build_matrix(src, dst)
    got = run_csr(torch, ns, *to_csr(k, c), src.size)
    assert ns.device_status() == 0
    assert got == oracle.stats_matrix(k, c).tolist() == oracle.stats(src, dst).tolist()


def test_csr_bad_input_is_reported(gpu):
    """A zero value, or a row_ptr that does not end at nnz, raises the device
    status; every read stays inside the arrays."""
    torch, ns = gpu
    say("csr invalid")
    src, dst = packets(33, 3000, 60)
    k, c = oracle.build_matrix(src, dst)
    rows, row_ptr, cols, vals = to_csr(k, c)
    zero = vals.copy()
    zero[zero.size // 2] = 0
    run_csr(torch, ns, rows, row_ptr, cols, zero, src.size)
    assert ns.device_status() == -1
    short = row_ptr.copy()
    short[-1] = short[-1] + 3
    run_csr(torch, ns, rows, short, cols, vals, src.size)
    assert ns.device_status() == -1
    assert ns.device_status() == 0  # reading clears the word


def test_csr_decreasing_row_pointers_are_reported(gpu):
    """Row pointers that run from 0 to nnz but decrease somewhere (so entries
    would land in other rows) raise the device status; so does a row pointer
    past nnz in the middle, and a decrease between two stored empty rows."""
    torch, ns = gpu
    say("csr decreasing row pointers")
    rows = np.array([5, 9], np.uint32)
    cols = np.array([1, 2], np.uint32)
    vals = np.array([1, 1], np.uint64)
    run_csr(torch, ns, rows, np.array([0, 3, 2], np.uint64), cols, vals, 2)
    assert ns.device_status() == -1
    run_csr(torch, ns, rows, np.array([0, 1, 2], np.uint64), cols, vals, 2)
    assert ns.device_status() == 0
    src, dst = packets(35, 4000, 80)
    k, c = oracle.build_matrix(src, dst)
    rows, row_ptr, cols, vals = to_csr(k, c, empty_rows=[7, 8, 0xFFFFFFF0])
    got = run_csr(torch, ns, rows, row_ptr, cols, vals, src.size)
    assert ns.device_status() == 0
    assert got == oracle.stats_matrix(k, c).tolist()
    for r in (1, rows.size // 2, rows.size - 1):
        bad = row_ptr.copy()
        bad[r] = bad[r + 1] + 1  # row_ptr[r] > row_ptr[r + 1]
        run_csr(torch, ns, rows, bad, cols, vals, src.size)
        assert ns.device_status() == -1, r


def test_csr_value_range_and_total_are_checked(gpu):
    """Values must lie in [1, 2^32) and sum to at most the caller's packet
    bound: a value of 2^32, two values whose 64-bit sum wraps around, a sum
    past the bound and keys out of order each raise the device status, while
    a bound equal to the sum is accepted."""
    torch, ns = gpu
    say("csr value range and packet total")
    src, dst = packets(34, 3000, 60)
    k, c = oracle.build_matrix(src, dst)
    rows, row_ptr, cols, vals = to_csr(k, c)
    assert c.max() > 1 and k.size < src.size
    big = vals.copy()
    big[1] = np.uint64(1 << 32)
    run_csr(torch, ns, rows, row_ptr, cols, big, src.size)
    assert ns.device_status() == -1
    wrap = vals.copy()
    wrap[0] = wrap[-1] = np.uint64(1 << 63)  # the sum wraps to below the bound
    run_csr(torch, ns, rows, row_ptr, cols, wrap, src.size)
    assert ns.device_status() == -1
    run_csr(torch, ns, rows, row_ptr, cols, vals, k.size)  # nnz <= bound < sum
    assert ns.device_status() == -1
    r = int(np.argmax(np.diff(row_ptr.astype(np.int64)) >= 2))
    e = int(row_ptr[r])
    assert row_ptr[r + 1] - row_ptr[r] >= 2
    swapped = cols.copy()
    swapped[e], swapped[e + 1] = cols[e + 1], cols[e]
    run_csr(torch, ns, rows, row_ptr, swapped, vals, src.size)
    assert ns.device_status() == -1
    got = run_csr(torch, ns, rows, row_ptr, cols, vals, int(c.sum()))
    assert ns.device_status() == 0
    assert got == oracle.stats_matrix(k, c).tolist()
