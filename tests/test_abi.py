"""libns.so loads on a host without a GPU and exports every symbol of include/ns.h."""
import ctypes
import os
import re

import pytest

from paper_2510_14050_amd import ns

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ns.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ns_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ns.LIB_PATH):
        pytest.skip("libns.so not built")
    return ns.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("ns_build_matrix", "ns_accumulate", "ns_stats", "ns_batch_stats",
              "ns_workspace_size", "ns_device_status", "ns_release_graphs", "ns_error_string"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(ns.EXPORTS)


def test_host_only_calls(lib):
    assert ns.version().startswith("libns")
    assert lib.ns_error_string(-2) == b"output capacity below the a-priori bound"
    small = ns.workspace_size(0, 1)
    big = ns.workspace_size(1 << 20, 64)
    assert 0 < small < big
    # workspace grows about linearly in packets (sort buffers + head arrays)
    assert ns.workspace_size(1 << 22, 1) > 4 * ns.workspace_size(1 << 20, 1) * 0.9
    bad = ctypes.c_uint64()
    assert lib.ns_workspace_size(10, 1, None) == -1
    assert lib.ns_workspace_size(10, 1, ctypes.byref(bad)) == 0


def test_host_argument_errors(lib):
    """Errors found on the host return before anything touches a device."""
    m = ns.MatrixView(0, 0, 0, 0, 0)
    assert lib.ns_build_matrix(None, None, 0, None, None, 0, None) == -1
    assert lib.ns_build_matrix(None, None, 5, ctypes.byref(m), None, 0, None) == -1
    fake = ns.MatrixView(256, 512, 768, 10, 10)
    # capacity below n
    assert lib.ns_build_matrix(ctypes.c_void_p(256), ctypes.c_void_p(256), 11,
                               ctypes.byref(fake), ctypes.c_void_p(256), 1 << 40, None) == -2
    # n beyond 2^32 - 1
    assert lib.ns_build_matrix(ctypes.c_void_p(256), ctypes.c_void_p(256), 1 << 32,
                               ctypes.byref(fake), ctypes.c_void_p(256), 1 << 40, None) == -6
    # misaligned / short workspace
    assert lib.ns_build_matrix(ctypes.c_void_p(256), ctypes.c_void_p(256), 4, ctypes.byref(fake),
                               ctypes.c_void_p(100), 1 << 40, None) == -3
    assert lib.ns_build_matrix(ctypes.c_void_p(256), ctypes.c_void_p(256), 4, ctypes.byref(fake),
                               ctypes.c_void_p(256), 16, None) == -3
    # accumulate: bad sign, aliasing, capacity, host-visible underflow
    a = ns.MatrixView(1024, 2048, 3072, 100, 100)
    b = ns.MatrixView(4096, 5120, 6144, 50, 50)
    c = ns.MatrixView(7168, 8192, 9216, 150, 0)
    ws = ctypes.c_void_p(1 << 20)
    assert lib.ns_accumulate(ctypes.byref(a), ctypes.byref(b), 0, ctypes.byref(c), ws, 1 << 40, None) == -1
    assert lib.ns_accumulate(ctypes.byref(a), ctypes.byref(b), 1, ctypes.byref(a), ws, 1 << 40, None) == -1
    small = ns.MatrixView(7168, 8192, 9216, 149, 0)
    assert lib.ns_accumulate(ctypes.byref(a), ctypes.byref(b), 1, ctypes.byref(small), ws, 1 << 40, None) == -2
    assert lib.ns_accumulate(ctypes.byref(b), ctypes.byref(a), -1, ctypes.byref(c), ws, 1 << 40, None) == -5
    # accumulate workspace: the merge needs a ticket and one word per merge tile
    need = ctypes.c_uint64()
    assert lib.ns_accumulate_workspace_size(100, 50, None) == -1
    assert lib.ns_accumulate_workspace_size(100, 50, ctypes.byref(need)) == 0
    assert 0 < need.value <= 4096
    big = ctypes.c_uint64()
    assert lib.ns_accumulate_workspace_size(1 << 31, 1 << 31, ctypes.byref(big)) == 0
    assert big.value >= 8 * ((1 << 32) // (256 * 8)) and big.value < (1 << 32) // 64
    full = ctypes.c_uint64()
    assert lib.ns_workspace_size(150, 1, ctypes.byref(full)) == 0 and full.value >= need.value
    assert lib.ns_accumulate(ctypes.byref(a), ctypes.byref(b), 1, ctypes.byref(c), ws,
                             need.value - 1, None) == -3
    assert lib.ns_accumulate(ctypes.byref(a), ctypes.byref(b), 1, ctypes.byref(c),
                             ctypes.c_void_p((1 << 20) + 8), 1 << 40, None) == -3
    # stats of a matrix holding 2^32 packets or more need fewer than 2^32 + 1 entries
    huge = ns.MatrixView(1024, 2048, 3072, (1 << 32) + 2, 1 << 33)
    assert lib.ns_stats(ctypes.byref(huge), ctypes.c_void_p(256), ws, 1 << 40, None) == -6
    # batch: bad tuning, capacity
    t = ns.tuning(sort_block=128)
    off = ctypes.c_void_p(256)
    assert lib.ns_batch_stats(off, off, off, 1, 10, off, None, None, None, ctypes.byref(t), ws,
                              1 << 40, None) == -1
    for bits in (1, 4, 7, 9, 10, 12, 16):  # digit widths other than 8 and 11
        t = ns.tuning(digit_bits=bits)
        assert lib.ns_batch_stats(off, off, off, 1, 10, off, None, None, None, ctypes.byref(t),
                                  ws, 1 << 40, None) == -1
    aggm = ns.MatrixView(1024, 2048, 3072, 9, 0)
    assert lib.ns_batch_stats(off, off, off, 1, 10, off, ctypes.byref(aggm), None, None, None, ws,
                              1 << 40, None) == -2
    # batch without per-window output: only with an aggregate, and no window matrices
    assert lib.ns_batch_stats(off, off, off, 4, 10, None, None, None, None, None, ws,
                              1 << 40, None) == -1
    agg_ok = ns.MatrixView(1024, 2048, 3072, 10, 0)
    wv = ns.BatchMatricesView(4096, 5120, 6144, 10)
    assert lib.ns_batch_stats(off, off, off, 4, 10, None, ctypes.byref(agg_ok), None,
                              ctypes.byref(wv), None, ws, 1 << 40, None) == -1
    assert lib.ns_batch_stats(off, off, off, 4, 10, None, ctypes.byref(aggm), None, None, None,
                              ws, 1 << 40, None) == -2
    # the batch total is below 2^32
    big_agg = ns.MatrixView(1024, 2048, 3072, 1 << 33, 0)
    assert lib.ns_batch_stats(off, off, off, 4, 1 << 32, None, ctypes.byref(big_agg), None, None,
                              None, ws, 1 << 40, None) == -6


def test_max_link_argument_errors(lib):
    assert lib.ns_max_link_packets(None, ctypes.c_void_p(256), None) == -1
    m = ns.MatrixView(1024, 2048, 3072, 10, 10)
    assert lib.ns_max_link_packets(ctypes.byref(m), None, None) == -1
    wv = ns.BatchMatricesView(1024, 2048, 3072, 100)
    off = ctypes.c_void_p(4096)
    # zero windows: nothing to do
    assert lib.ns_batch_max_link_packets(ctypes.byref(wv), off, 0, 100, ctypes.c_void_p(256), None) == 0
    assert lib.ns_batch_max_link_packets(None, off, 4, 100, ctypes.c_void_p(256), None) == -1
    assert lib.ns_batch_max_link_packets(ctypes.byref(wv), None, 4, 100, ctypes.c_void_p(256), None) == -1
    # capacity below the scanned positions
    assert lib.ns_batch_max_link_packets(ctypes.byref(wv), off, 4, 101, ctypes.c_void_p(256), None) == -2


def test_streamed_build_argument_errors(lib):
    """ns_build_matrix_streamed rejects bad arguments before any device call."""
    out = ns.MatrixView(1024, 2048, 3072, 100, 0)
    ws = ctypes.c_void_p(1 << 20)
    host = ctypes.c_void_p(4096)
    size = ctypes.c_uint64()
    assert lib.ns_stream_workspace_size(0, 100, ctypes.byref(size)) == -1
    assert lib.ns_stream_workspace_size(10, 100, None) == -1
    assert lib.ns_stream_workspace_size(1000, 100, ctypes.byref(size)) == 0
    small = size.value
    assert lib.ns_stream_workspace_size(1000, 1 << 20, ctypes.byref(size)) == 0
    assert size.value > small + 16 * ((1 << 20) - 100) * 0.99  # second aggregate buffer
    args = lambda n, batch, o, w, nbytes: (host, host, n, batch, o, w, nbytes, None, None)
    assert lib.ns_build_matrix_streamed(*args(10, 4, None, ws, 1 << 40)) == -1
    assert lib.ns_build_matrix_streamed(None, None, 10, 4, ctypes.byref(out), ws, 1 << 40, None, None) == -1
    assert lib.ns_build_matrix_streamed(*args(10, 0, ctypes.byref(out), ws, 1 << 40)) == -1
    assert lib.ns_build_matrix_streamed(*args(10, 1 << 32, ctypes.byref(out), ws, 1 << 40)) == -6
    tiny = ns.MatrixView(1024, 2048, 3072, 3, 0)  # below the first sub-partition
    assert lib.ns_build_matrix_streamed(*args(10, 4, ctypes.byref(tiny), ws, 1 << 40)) == -2
    assert lib.ns_build_matrix_streamed(*args(10, 4, ctypes.byref(out), ctypes.c_void_p(100), 1 << 40)) == -3
    assert lib.ns_build_matrix_streamed(*args(10, 4, ctypes.byref(out), ws, 64)) == -3


def test_stats_csr_argument_errors(lib):
    """ns_stats_csr rejects bad arguments before any device call."""
    size = ctypes.c_uint64()
    assert lib.ns_stats_csr_workspace_size(100, None) == -1
    assert lib.ns_stats_csr_workspace_size(100, ctypes.byref(size)) == 0
    assert size.value >= 16 * 100
    p = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    # rows, row_ptr, nrows, cols, vals, nnz, packets, out, ws, ws_bytes, stream
    assert lib.ns_stats_csr(p, p, 1, p, p, 4, 4, None, ws, 1 << 40, None) == -1   # no output
    assert lib.ns_stats_csr(p, None, 1, p, p, 4, 4, p, ws, 1 << 40, None) == -1   # no row_ptr
    assert lib.ns_stats_csr(p, p, 0, p, p, 4, 4, p, ws, 1 << 40, None) == -1      # entries, no rows
    assert lib.ns_stats_csr(p, p, 1, None, p, 4, 4, p, ws, 1 << 40, None) == -1
    assert lib.ns_stats_csr(p, p, 1, p, p, 4, 3, p, ws, 1 << 40, None) == -1      # packets < nnz
    assert lib.ns_stats_csr(p, p, 1, p, p, 4, 1 << 32, p, ws, 1 << 40, None) == -6
    assert lib.ns_stats_csr(p, p, 1, p, p, 4, 4, p, ctypes.c_void_p(100), 1 << 40, None) == -3
    assert lib.ns_stats_csr(p, p, 1, p, p, 4, 4, p, ws, 64, None) == -3
