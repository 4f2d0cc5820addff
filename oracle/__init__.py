"""CPU oracle for the eight network quantities and for union-add.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may import this package; the product path never does. The arithmetic
lives in ``ns_oracle.cpp`` (plain C++, std::map and std::sort, compiled with
g++); this module only builds it and marshals numpy arrays. It shares no code
with the HIP library.

Statistic order (Table I plus the row- and column-sum maxima):
valid packets, unique links, unique sources, unique destinations,
max source packets, max source fan-out, max destination packets,
max destination fan-in.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ns_oracle.cpp")
LIB = os.path.join(HERE, "libns_oracle.so")

STAT_NAMES = (
    "valid_packets", "unique_links", "unique_sources", "unique_destinations",
    "max_source_packets", "max_source_fanout", "max_destination_packets",
    "max_destination_fanin",
)

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no GPU code involved)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", SRC, "-o", tmp],
                       check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        U = ctypes.c_uint64
        lib.oracle_stats_map.argtypes = [P, P, U, P]
        lib.oracle_stats_map.restype = None
        lib.oracle_build.argtypes = [P, P, U, P, P]
        lib.oracle_build.restype = U
        lib.oracle_stats_matrix.argtypes = [P, P, U, P]
        lib.oracle_stats_matrix.restype = None
        lib.oracle_stats_packets.argtypes = [P, P, U, P]
        lib.oracle_stats_packets.restype = None
        lib.oracle_stats_windows.argtypes = [P, P, P, U, P]
        lib.oracle_stats_windows.restype = None
        lib.oracle_accumulate.argtypes = [P, P, U, P, P, U, ctypes.c_int, P, P]
        lib.oracle_accumulate.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _u32(a) -> np.ndarray:
    a = np.asarray(a)
    if a.dtype != np.uint32:
        a = a.astype(np.uint64).astype(np.uint32) if a.dtype.kind in "iu" else a.astype(np.uint32)
    return np.ascontiguousarray(a)


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def stats_map(src, dst) -> np.ndarray:
    """The eight quantities by the std::map route (definitions)."""
    s, d = _u32(src), _u32(dst)
    assert s.size == d.size
    out = np.zeros(8, np.uint64)
    _load().oracle_stats_map(_ptr(s), _ptr(d), s.size, _ptr(out))
    return out


def build_matrix(src, dst):
    """Sorted COO (keys = src<<32|dst strictly increasing, counts >= 1)."""
    s, d = _u32(src), _u32(dst)
    assert s.size == d.size
    keys = np.empty(max(s.size, 1), np.uint64)
    counts = np.empty(max(s.size, 1), np.uint64)
    nnz = _load().oracle_build(_ptr(s), _ptr(d), s.size, _ptr(keys), _ptr(counts))
    return keys[:nnz].copy(), counts[:nnz].copy()


def stats_matrix(keys, counts) -> np.ndarray:
    k, c = _u64(keys), _u64(counts)
    out = np.zeros(8, np.uint64)
    _load().oracle_stats_matrix(_ptr(k), _ptr(c), k.size, _ptr(out))
    return out


def stats(src, dst) -> np.ndarray:
    """The eight quantities by the sort route."""
    s, d = _u32(src), _u32(dst)
    out = np.zeros(8, np.uint64)
    _load().oracle_stats_packets(_ptr(s), _ptr(d), s.size, _ptr(out))
    return out


def stats_windows(src, dst, offsets) -> np.ndarray:
    """Per-window quantities, shape (W, 8)."""
    s, d, o = _u32(src), _u32(dst), _u64(offsets)
    W = o.size - 1
    out = np.zeros((max(W, 0), 8), np.uint64)
    if W > 0:
        _load().oracle_stats_windows(_ptr(s), _ptr(d), _ptr(o), W, _ptr(out))
    return out


def accumulate(keys_a, counts_a, keys_b, counts_b, sign: int = 1):
    """A + sign*B as sorted COO; raises ValueError when subtraction underflows."""
    ka, ca, kb, cb = _u64(keys_a), _u64(counts_a), _u64(keys_b), _u64(counts_b)
    cap = max(ka.size + kb.size, 1)
    kc = np.empty(cap, np.uint64)
    cc = np.empty(cap, np.uint64)
    nnz = _load().oracle_accumulate(_ptr(ka), _ptr(ca), ka.size, _ptr(kb), _ptr(cb), kb.size,
                                    int(sign), _ptr(kc), _ptr(cc))
    if nnz < 0:
        raise ValueError("subtraction below zero")
    return kc[:nnz].copy(), cc[:nnz].copy()


def max_link_packets(src, dst) -> int:
    """Largest link count max_ij A(i,j) (Sec. IV, "Analytics and Operations":
    maximum link counts): the largest count of the sorted COO, 0 when empty."""
    _, counts = build_matrix(src, dst)
    return int(counts.max()) if counts.size else 0


def max_link_packets_windows(src, dst, offsets) -> np.ndarray:
    """Per-window largest link count, shape (W,)."""
    o = _u64(offsets)
    s, d = _u32(src), _u32(dst)
    return np.array([max_link_packets(s[int(o[w]):int(o[w + 1])], d[int(o[w]):int(o[w + 1])])
                     for w in range(o.size - 1)], np.uint64)

