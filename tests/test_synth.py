"""The input generator: deterministic, back-end independent, and shaped as
stated (distinct pool, Zipf skew, scanner/sink counts, size laws)."""
import numpy as np
import pytest

from paper_2510_14050_amd import synth


def test_numpy_and_torch_back_ends_agree():
    torch = pytest.importorskip("torch")
    for wl in (synth.one_window(1 << 12), synth.aggregate_2p30(num=3, n=1 << 12)):
        for w in range(wl.num_windows):
            s, d = wl.window(w)
            ts, td = wl.window(w, device="cpu")
            assert np.array_equal(synth.as_u32(ts), s)
            assert np.array_equal(synth.as_u32(td), d)


def test_windows_depend_only_on_their_index():
    a = synth.Workload("t", 3, 1 << 10, 1.2, 1.2, np.array([100, 200, 300], np.int64))
    b = synth.Workload("t", 3, 1 << 10, 1.2, 1.2, np.array([5, 200, 7], np.int64))
    assert np.array_equal(a.window(1)[0], b.window(1)[0])
    assert not np.array_equal(a.window(0)[0][:5], a.window(1)[0][:5])


def test_pool_is_distinct_and_zipf_is_skewed():
    pool = synth.distinct_addresses(4, 1 << 14)
    assert np.unique(pool).size == pool.size == 1 << 14
    wl = synth.Workload("t", 4, 1 << 14, 1.2, 1.2, np.array([1 << 16], np.int64))
    s, d = wl.window(0)
    _, c = np.unique(s, return_counts=True)
    # rank 1 of Zipf(1.2) over 2^14 ranks carries about 1/zeta-ish mass (~18%)
    assert 0.12 < c.max() / s.size < 0.25
    # the top source is not the top destination (ranks are permuted for dst)
    _, cd = np.unique(d, return_counts=True)
    assert np.unique(s)[c.argmax()] != np.unique(d)[cd.argmax()]


def test_scanner_and_sink_shape():
    wl = synth.aggregate_2p30(num=4, n=1 << 14)
    m = wl.scan_count(1 << 14)
    assert m == round(0.01 * (1 << 14))
    targets = set()
    for w in range(4):
        s, d = wl.window(w)
        assert (s == wl.scanner).sum() == m
        assert (d == wl.sink).sum() == m
        targets.update(d[s == wl.scanner].tolist())
    # round robin over the 2^16 targets: all distinct so far
    assert len(targets) == 4 * m
    assert wl.scanner not in wl._pool and wl.sink not in wl._pool


def test_size_laws():
    u = synth.uneven1024()
    assert u.sizes.min() >= 1 << 12 and u.sizes.max() <= 1 << 17
    assert abs(np.log2(u.sizes).mean() - 14.5) < 0.2
    sv = synth.serving(num=2000)
    assert sv.sizes.min() >= 1 << 10 and sv.sizes.max() <= 1 << 17
    gaps = np.diff(sv.arrivals)
    assert abs(gaps.mean() - 1 / 2000) < 0.1 / 2000
