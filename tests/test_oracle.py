"""Pins for the CPU oracle (runs without a GPU).

The paper prints no statistic values, so the oracle is pinned by hand-worked
fixtures (tests/golden), brute-force enumeration on tiny windows, closed forms,
invariants, symmetries and the algebra of aggregation. A second group of tests
plants mistakes into copies of the oracle source and checks that the pins
catch each of them.
"""
import glob
import itertools
import os
import random
import shutil
import subprocess

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_fixture(path):
    src, dst, expect = [], [], None
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        if line.startswith("expect:"):
            expect = [int(x) for x in line.split(":", 1)[1].split()]
            continue
        a, b = line.split()
        src.append(int(a, 0))
        dst.append(int(b, 0))
    return np.array(src, np.uint32), np.array(dst, np.uint32), np.array(expect, np.uint64)


def distinct_u32(rng, n):
    """n distinct random uint32 values (rejection of repeats)."""
    out = np.empty(0, np.uint32)
    while out.size < n:
        cand = rng.integers(0, 2**32, 2 * n + 8, dtype=np.uint64).astype(np.uint32)
        _, first = np.unique(np.concatenate([out, cand]), return_index=True)
        out = np.concatenate([out, cand])[np.sort(first)]
    return out[:n]


def brute_force(src, dst):
    """Enumerate every (i, j) of the observed addresses and count packets by a
    full scan; then apply the definitions. Quadratic, for tiny windows only."""
    pairs = list(zip([int(x) for x in src], [int(x) for x in dst]))
    I = sorted(set(p[0] for p in pairs))
    J = sorted(set(p[1] for p in pairs))
    A = {}
    for i in I:
        for j in J:
            a = sum(1 for p in pairs if p[0] == i and p[1] == j)
            if a:
                A[(i, j)] = a
    row_pk = [sum(A.get((i, j), 0) for j in J) for i in I]
    row_nz = [sum(1 for j in J if (i, j) in A) for i in I]
    col_pk = [sum(A.get((i, j), 0) for i in I) for j in J]
    col_nz = [sum(1 for i in I if (i, j) in A) for j in J]
    return np.array([
        sum(A.values()), len(A),
        sum(1 for x in row_pk if x > 0), sum(1 for x in col_pk if x > 0),
        max(row_pk, default=0), max(row_nz, default=0),
        max(col_pk, default=0), max(col_nz, default=0)], np.uint64), A


ROUTES = ("map", "sort", "matrix")


def route_stats(oracle, route, s, d):
    if route == "map":
        return oracle.stats_map(s, d)
    if route == "sort":
        return oracle.stats(s, d)
    k, c = oracle.build_matrix(s, d)
    return oracle.stats_matrix(k, c)


# --------------------------------------------------------------------------
# hand-worked fixtures
# --------------------------------------------------------------------------

FIXTURES = [p for p in sorted(glob.glob(os.path.join(GOLDEN, "*.txt")))
            if not p.endswith("README.txt")]


@pytest.mark.parametrize("path", FIXTURES, ids=[os.path.basename(p) for p in FIXTURES])
@pytest.mark.parametrize("route", ROUTES)
def test_golden_fixture(oracle_mod, path, route):
    s, d, expect = read_fixture(path)
    got = route_stats(oracle_mod, route, s, d)
    assert got.tolist() == expect.tolist(), os.path.basename(path)


# --------------------------------------------------------------------------
# brute force on tiny windows with forced collisions
# --------------------------------------------------------------------------

EDGE = [0, 1, 0x7FFFFFFF, 0x80000000, 0x80000001, 0xFFFFFFFE, 0xFFFFFFFF]
addr = st.one_of(st.sampled_from(EDGE), st.integers(0, 2**32 - 1))


@settings(max_examples=150, deadline=None)
@given(st.lists(addr, min_size=1, max_size=8, unique=True),
       st.lists(addr, min_size=1, max_size=8, unique=True),
       st.lists(st.tuples(st.integers(0, 7), st.integers(0, 7)), max_size=96))
def test_brute_force_tiny(oracle_mod, pool_s, pool_d, picks):
    s = np.array([pool_s[a % len(pool_s)] for a, _ in picks], np.uint32)
    d = np.array([pool_d[b % len(pool_d)] for _, b in picks], np.uint32)
    expect, A = brute_force(s, d)
    for route in ROUTES:
        assert route_stats(oracle_mod, route, s, d).tolist() == expect.tolist(), route
    keys, counts = oracle_mod.build_matrix(s, d)
    want = sorted(((i << 32) | j, a) for (i, j), a in A.items())
    assert keys.tolist() == [k for k, _ in want]
    assert counts.tolist() == [a for _, a in want]


# --------------------------------------------------------------------------
# closed forms (tuple = the eight quantities in library order)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("route", ROUTES)
@pytest.mark.parametrize("n", [1, 2, 7, 1000])
def test_identical_pairs(oracle_mod, route, n):
    s = np.full(n, 0xC0A80001, np.uint32)
    d = np.full(n, 0x0A000001, np.uint32)
    assert route_stats(oracle_mod, route, s, d).tolist() == [n, 1, 1, 1, n, 1, n, 1]


@pytest.mark.parametrize("route", ROUTES)
@pytest.mark.parametrize("a,b,r", [(1, 1, 1), (3, 5, 2), (7, 2, 3), (16, 9, 1)])
def test_grid(oracle_mod, route, a, b, r):
    rng = np.random.default_rng(a * 100 + b * 10 + r)
    S = distinct_u32(rng, a)
    D = distinct_u32(rng, b)
    s = np.repeat(np.repeat(S, b), r)
    d = np.repeat(np.tile(D, a), r)
    perm = rng.permutation(s.size)
    got = route_stats(oracle_mod, route, s[perm], d[perm])
    assert got.tolist() == [a * b * r, a * b, a, b, b * r, b, a * r, a]


@pytest.mark.parametrize("route", ROUTES)
def test_matching(oracle_mod, route):
    rng = np.random.default_rng(5)
    n = 5000
    s = distinct_u32(rng, n)
    d = distinct_u32(rng, n)
    assert route_stats(oracle_mod, route, s, d).tolist() == [n, n, n, n, 1, 1, 1, 1]


@pytest.mark.parametrize("route", ROUTES)
@pytest.mark.parametrize("m", [1, 2, 300])
def test_scanner_and_sink(oracle_mod, route, m):
    rng = np.random.default_rng(m)
    T = distinct_u32(rng, m)
    s = np.full(m, 0xDEADBEEF, np.uint32)
    assert route_stats(oracle_mod, route, s, T).tolist() == [m, m, 1, m, m, m, 1, 1]
    assert route_stats(oracle_mod, route, T, s).tolist() == [m, m, m, 1, 1, 1, m, m]


# --------------------------------------------------------------------------
# invariants and symmetries on generated Zipf traffic
# --------------------------------------------------------------------------

def zipf_window(seed, n, pool=512, s=1.2):
    from paper_2510_14050_amd import synth
    wl = synth.Workload("t", seed, pool, s, s + 0.1, np.array([n], np.int64))
    return wl.window(0)


def check_invariants(st8):
    v, links, ns, nd, msp, mfo, mdp, mfi = [int(x) for x in st8]
    assert links <= v
    assert links >= max(mfo, mfi)
    if v:
        assert max(ns, nd) <= links <= ns * nd
        assert msp * ns >= v and mdp * nd >= v
    assert mfo <= min(nd, msp)
    assert mfi <= min(ns, mdp)


@pytest.mark.parametrize("seed,n", [(11, 1), (12, 100), (13, 4096), (14, 1 << 15)])
def test_invariants_and_row_col_sums(oracle_mod, seed, n):
    s, d = zipf_window(seed, n)
    st8 = oracle_mod.stats(s, d)
    check_invariants(st8)
    keys, counts = oracle_mod.build_matrix(s, d)
    # sum of row packet counts = sum of column packet counts = valid packets
    rows = keys >> np.uint64(32)
    cols = keys & np.uint64(0xFFFFFFFF)
    _, rinv = np.unique(rows, return_inverse=True)
    _, cinv = np.unique(cols, return_inverse=True)
    assert int(np.bincount(rinv, weights=counts.astype(np.float64)).sum()) == int(st8[0]) == n
    assert int(np.bincount(cinv, weights=counts.astype(np.float64)).sum()) == n
    assert int(counts.sum()) == n
    assert np.all(keys[1:] > keys[:-1])


@pytest.mark.parametrize("route", ROUTES)
def test_symmetries(oracle_mod, route):
    s, d = zipf_window(21, 20000, pool=2048)
    base = route_stats(oracle_mod, route, s, d)
    # transpose swaps (sources, destinations), (max src pk, max dst pk), (fan-out, fan-in)
    t = route_stats(oracle_mod, route, d, s)
    assert t.tolist() == base[[0, 1, 3, 2, 6, 7, 4, 5]].tolist()
    # packet order does not matter
    perm = np.random.default_rng(1).permutation(s.size)
    assert route_stats(oracle_mod, route, s[perm], d[perm]).tolist() == base.tolist()
    # any bijection of the address space leaves every quantity unchanged
    flip = np.uint32(0x80000000)
    assert route_stats(oracle_mod, route, s ^ flip, d ^ flip).tolist() == base.tolist()
    u = np.unique(np.concatenate([s, d]))
    img = distinct_u32(np.random.default_rng(2), u.size)
    f = lambda x: img[np.searchsorted(u, x)]
    assert route_stats(oracle_mod, route, f(s), f(d)).tolist() == base.tolist()


def test_routes_agree_on_zipf(oracle_mod):
    for seed, n in [(31, 1 << 12), (32, 1 << 16)]:
        s, d = zipf_window(seed, n, pool=1 << 14)
        a = oracle_mod.stats_map(s, d)
        assert oracle_mod.stats(s, d).tolist() == a.tolist()
        k, c = oracle_mod.build_matrix(s, d)
        assert oracle_mod.stats_matrix(k, c).tolist() == a.tolist()


def test_windows_helper(oracle_mod):
    s, d = zipf_window(41, 3000)
    off = np.array([0, 0, 1000, 1001, 3000], np.uint64)
    got = oracle_mod.stats_windows(s, d, off)
    for w in range(4):
        a, b = int(off[w]), int(off[w + 1])
        assert got[w].tolist() == oracle_mod.stats_map(s[a:b], d[a:b]).tolist()


# --------------------------------------------------------------------------
# aggregation algebra
# --------------------------------------------------------------------------

def test_union_add_algebra(oracle_mod):
    s1, d1 = zipf_window(51, 5000, pool=300)
    s2, d2 = zipf_window(52, 7000, pool=300)
    s3, d3 = zipf_window(53, 100, pool=300)
    A = oracle_mod.build_matrix(s1, d1)
    B = oracle_mod.build_matrix(s2, d2)
    C = oracle_mod.build_matrix(s3, d3)
    AB = oracle_mod.accumulate(*A, *B, 1)
    BA = oracle_mod.accumulate(*B, *A, 1)
    # aggregate of matrices = matrix of the concatenated packets
    cat = oracle_mod.build_matrix(np.concatenate([s1, s2]), np.concatenate([d1, d2]))
    for x, y in zip(AB, cat):
        assert x.tolist() == y.tolist()
    for x, y in zip(AB, BA):
        assert x.tolist() == y.tolist()
    ABC1 = oracle_mod.accumulate(*AB, *C, 1)
    ABC2 = oracle_mod.accumulate(*A, *oracle_mod.accumulate(*B, *C, 1), 1)
    for x, y in zip(ABC1, ABC2):
        assert x.tolist() == y.tolist()
    # subtraction is the exact inverse and drops zeros
    back = oracle_mod.accumulate(*AB, *B, -1)
    for x, y in zip(back, A):
        assert x.tolist() == y.tolist()
    empty = oracle_mod.accumulate(*A, *A, -1)
    assert empty[0].size == 0
    # valid packets add up; stats of the sum = stats of the concatenation
    assert int(oracle_mod.stats_matrix(*AB)[0]) == 12000
    with pytest.raises(ValueError):
        oracle_mod.accumulate(*A, *AB, -1)


def test_brute_force_union(oracle_mod):
    rng = random.Random(7)
    for _ in range(30):
        la = [(rng.randrange(4), rng.randrange(4)) for _ in range(rng.randrange(12))]
        lb = [(rng.randrange(4), rng.randrange(4)) for _ in range(rng.randrange(12))]
        A = oracle_mod.build_matrix([p[0] for p in la], [p[1] for p in la])
        B = oracle_mod.build_matrix([p[0] for p in lb], [p[1] for p in lb])
        k, c = oracle_mod.accumulate(*A, *B, 1)
        want = {}
        for i, j in la + lb:
            want[(i << 32) | j] = want.get((i << 32) | j, 0) + 1
        assert list(zip(k.tolist(), c.tolist())) == sorted(want.items())


# --------------------------------------------------------------------------
# planted mistakes: each mutant of the oracle source must fail a pin
# --------------------------------------------------------------------------

MUTANTS = [
    # (description, original text, replacement)
    ("fan-out counts packets", "out[5] = std::max(out[5], q - p);",
     "out[5] = std::max(out[5], packets);"),
    ("rows keyed by destination", "const uint64_t i = keys[p] >> 32;",
     "const uint64_t i = keys[p] & 0xFFFFFFFFu;"),
    ("column count off by one", "out[3] += 1;\n    out[6]", "out[3] += (p > 0);\n    out[6]"),
    ("column sums drop the count", "packets += col[q++].second;",
     "packets += 1 + 0 * col[q++].second;"),
    ("transposed key", "k[p] = (uint64_t(src[p]) << 32) | uint64_t(dst[p]);",
     "k[p] = (uint64_t(dst[p]) << 32) | uint64_t(src[p]);"),
    ("valid counts links", "out[0] += packets;", "out[0] += q - p;"),
    ("signed key order", "std::sort(k.begin(), k.end());",
     "std::sort(k.begin(), k.end(), [](uint64_t a, uint64_t b) { return int64_t(a) < int64_t(b); });"),
    ("fan-in counts packets", "out[7] = std::max(out[7], q - p);",
     "out[7] = std::max(out[7], packets);"),
    ("last row dropped", "while (q < nnz && (keys[q] >> 32) == i) packets += counts[q++];",
     "while (q < nnz && (keys[q] >> 32) == i) packets += counts[q++];\n    if (q == nnz) break;"),
]


def _pins_hold(lib_path):
    """Run a compact subset of the pins against a compiled oracle library."""
    import ctypes
    lib = ctypes.CDLL(lib_path)
    P, U = ctypes.c_void_p, ctypes.c_uint64
    lib.oracle_stats_packets.argtypes = [P, P, U, P]
    lib.oracle_build.argtypes = [P, P, U, P, P]
    lib.oracle_build.restype = U

    def run(s, d):
        s = np.ascontiguousarray(s, np.uint32)
        d = np.ascontiguousarray(d, np.uint32)
        out = np.zeros(8, np.uint64)
        lib.oracle_stats_packets(s.ctypes.data_as(P), d.ctypes.data_as(P), s.size,
                                 out.ctypes.data_as(P))
        return out.tolist()

    for path in sorted(glob.glob(os.path.join(GOLDEN, "*.txt"))):
        if path.endswith("README.txt"):
            continue
        s, d, e = read_fixture(path)
        if run(s, d) != e.tolist():
            return False
    S = np.array([5, 9, 0x90000000], np.uint32)
    D = np.array([1, 2, 3, 4, 0x80000007], np.uint32)
    s = np.repeat(np.repeat(S, 5), 2)
    d = np.repeat(np.tile(D, 3), 2)
    if run(s, d) != [30, 15, 3, 5, 10, 5, 6, 3]:
        return False
    # the built matrix is in unsigned key order
    s, d, _ = read_fixture(os.path.join(GOLDEN, "sign_boundary.txt"))
    keys = np.zeros(s.size, np.uint64)
    counts = np.zeros(s.size, np.uint64)
    nnz = lib.oracle_build(s.ctypes.data_as(P), d.ctypes.data_as(P), s.size,
                           keys.ctypes.data_as(P), counts.ctypes.data_as(P))
    if not (nnz == 4 and np.all(keys[1:nnz] > keys[:nnz - 1])):
        return False
    return True


def _pins_hold_isolated(lib_path):
    """_pins_hold in a child process, so a mutant that loops forever counts as caught."""
    import sys
    code = ("import sys; sys.path.insert(0, %r); import test_oracle as t; "
            "sys.exit(0 if t._pins_hold(%r) else 1)" % (os.path.dirname(__file__), lib_path))
    try:
        r = subprocess.run([sys.executable, "-c", code], timeout=30, capture_output=True)
    except subprocess.TimeoutExpired:
        return False
    return r.returncode == 0


def test_planted_mistakes_are_caught(tmp_path, oracle_mod):
    src = open(oracle_mod.SRC).read()
    assert _pins_hold_isolated(oracle_mod.LIB)
    for desc, old, new in MUTANTS:
        assert old in src, desc
        mutated = tmp_path / "mut.cpp"
        mutated.write_text(src.replace(old, new, 1))
        lib = tmp_path / f"mut_{abs(hash(desc))}.so"
        subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", str(mutated), "-o",
                        str(lib)], check=True)
        assert not _pins_hold_isolated(str(lib)), f"planted mistake not caught: {desc}"
