"""ns_accumulate_noalloc (the union-add for callers that cannot allocate device
memory) against ns_accumulate with a caller workspace: the same sorted COO
output bit for bit, on two calls in a row on the library's one scratch array,
the second with smaller inputs; and the oracle's union on both."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2510_14050_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def matrix_of(torch, ns, src, dst):
    n = src.size
    m = ns.Matrix(n)
    ws = ns.Workspace(n, 1)
    ns.build_matrix(torch.from_numpy(src.view(np.int32)).cuda(),
                    torch.from_numpy(dst.view(np.int32)).cuda(), m, ws)
    return m


def window(seed, n, pool):
    wl = synth.Workload("noalloc_t", seed, pool, 1.2, 1.3, np.array([n], np.int64))
    return wl.window(0)


@pytest.mark.parametrize("sign", [1, -1])
def test_noalloc_matches_workspace_call(sign):
    import torch
    from paper_2510_14050_amd import ns
    lib = ns.load()
    cases = [(3, 700_000, 150_000, 1 << 14), (4, 9_000, 2_500, 1 << 10)]  # second call smaller
    for seed, na_pk, nb_pk, pool in cases:
        say("noalloc union", "add" if sign > 0 else "subtract", na_pk, nb_pk)
        sa, da = window(seed, na_pk, pool)
        sb, db = window(seed + 100, nb_pk, pool)
        if sign < 0:  # subtract a part of A: its first nb_pk packets
            sb, db = sa[:nb_pk].copy(), da[:nb_pk].copy()
        A = matrix_of(torch, ns, sa, da)
        B = matrix_of(torch, ns, sb, db)
        cap = na_pk + (nb_pk if sign > 0 else 0)
        want_m = ns.Matrix(cap)
        ns.accumulate(A, B, sign, want_m, ns.MergeWorkspace(na_pk, nb_pk))
        got_m = ns.Matrix(cap)
        # fill the output with a marker so stale entries would show
        got_m.keys.fill_(-7)
        got_m.counts.fill_(-7)
        a, b, c = A.view(), B.view(), got_m.view()
        rc = lib.ns_accumulate_noalloc(ctypes.byref(a), ctypes.byref(b), sign, ctypes.byref(c),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0, rc
        assert c.packets == want_m.packets
        torch.cuda.synchronize()
        assert ns.device_status() == 0
        k, cnt = got_m.numpy()
        wk, wc = want_m.numpy()
        assert np.array_equal(k, wk) and np.array_equal(cnt, wc)
        ok, oc = oracle.build_matrix(sa, da)
        bk, bc = oracle.build_matrix(sb, db)
        ek, ec = oracle.accumulate(ok, oc, bk, bc, sign)
        assert np.array_equal(k, ek) and np.array_equal(cnt, ec)


def test_noalloc_rejects_beyond_its_maximum():
    from paper_2510_14050_amd import ns
    lib = ns.load()
    big = ns.ACCUMULATE_NOALLOC_MAX_ENTRIES
    a = ns.MatrixView(1024, 2048, 3072, big, big)
    b = ns.MatrixView(4096, 5120, 6144, 1, 1)
    c = ns.MatrixView(7168, 8192, 9216, big + 1, 0)
    assert lib.ns_accumulate_noalloc(ctypes.byref(a), ctypes.byref(b), 1, ctypes.byref(c),
                                     None) == -6
