"""Rolling aggregate in device hash tables (ns_rolling_*) against the oracle:
after every add / remove the eight quantities equal the oracle's on the
multiset of packets currently in the aggregate."""
import sys

import numpy as np
import pytest

import oracle
from paper_2510_14050_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def windows(n, seed, lo=6, hi=11, pool=300):
    sizes = synth.log_uniform_sizes(seed, n, lo, hi)
    wl = synth.Workload("roll_t", seed, pool, 1.2, 1.3, sizes)
    out = [wl.window(w) for w in range(n)]
    # plant the all-ones key (src = dst = 255.255.255.255) and extreme addresses
    s, d = out[1]
    s[:3], d[:3] = 0xFFFFFFFF, 0xFFFFFFFF
    s[3], d[3] = 0, 0xFFFFFFFF
    return out


@pytest.mark.parametrize("link_slots,addr_slots", [(1 << 14, 1 << 12), (1 << 20, 1 << 18)])
def test_rolling_matches_oracle(link_slots, addr_slots):
    import torch
    from paper_2510_14050_amd import ns
    say("rolling", link_slots, addr_slots)
    ring = 5
    wins = windows(24, 3)
    ws = ns.Workspace(1 << 11, 1)
    mats = []
    for s, d in wins:
        m = ns.Matrix(s.size)
        ns.build_matrix(torch.from_numpy(s.view(np.int32)).cuda(),
                        torch.from_numpy(d.view(np.int32)).cuda(), m, ws)
        mats.append(m)
    states = [ns.RollingState(link_slots, addr_slots), ns.RollingState(link_slots, addr_slots)]
    cur = 0
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    occ = torch.zeros(3, dtype=torch.int64, device="cuda")
    ones = (1 << 64) - 1  # the all-ones link is counted outside the table

    def keys(j):
        s, d = wins[j]
        return set(((s.astype(np.uint64) << np.uint64(32)) | d.astype(np.uint64)).tolist()) - {ones}
    taken = [set(), set(), set()]  # keys that took a slot since the clear / compaction
    for k in range(len(wins)):
        old = mats[k - ring] if k >= ring else None
        ns.rolling_update(states[cur], mats[k], old, out)
        taken[0] |= keys(k)
        taken[1] |= set(wins[k][0].tolist())
        taken[2] |= set(wins[k][1].tolist())
        lo = max(0, k - ring + 1)
        if k % 7 == 6:  # compaction keeps everything
            ns.rolling_compact(states[cur], states[1 - cur])
            cur = 1 - cur
            taken = [set().union(*(keys(j) for j in range(lo, k + 1))),
                     set(np.concatenate([wins[j][0] for j in range(lo, k + 1)]).tolist()),
                     set(np.concatenate([wins[j][1] for j in range(lo, k + 1)]).tolist())]
        ns.rolling_occupancy(states[cur], occ)
        torch.cuda.synchronize()
        want = oracle.stats(np.concatenate([wins[j][0] for j in range(lo, k + 1)]),
                            np.concatenate([wins[j][1] for j in range(lo, k + 1)]))
        assert ns.stats_numpy(out).tolist() == want.tolist(), k
        assert occ.cpu().tolist() == [len(t) for t in taken], k
    assert ns.device_status() == 0
    # remove everything that is left: the empty aggregate
    for k in range(len(wins) - ring, len(wins)):
        ns.rolling_update(states[cur], None, mats[k], out)
    torch.cuda.synchronize()
    assert ns.stats_numpy(out).tolist() == [0] * 8
    assert ns.device_status() == 0


def test_rolling_errors():
    import torch
    from paper_2510_14050_amd import ns
    say("rolling errors")
    wins = windows(3, 9, lo=9, hi=10, pool=5000)
    ws = ns.Workspace(1 << 10, 1)
    mats = []
    for s, d in wins:
        m = ns.Matrix(s.size)
        ns.build_matrix(torch.from_numpy(s.view(np.int32)).cuda(),
                        torch.from_numpy(d.view(np.int32)).cuda(), m, ws)
        mats.append(m)
    out = torch.zeros(8, dtype=torch.int64, device="cuda")
    st = ns.RollingState(1 << 12, 1 << 12)
    ns.rolling_update(st, mats[0], None, out)
    ns.rolling_update(st, None, mats[1], out)      # never added
    assert ns.device_status() == -5
    tiny = ns.RollingState(64, 64)                  # far fewer slots than entries
    ns.rolling_update(tiny, mats[2], None, out)
    assert ns.device_status() == -2
    assert ns.device_status() == 0
