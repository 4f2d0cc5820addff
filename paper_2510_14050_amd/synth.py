"""Seeded synthetic traffic: windows of (source, destination) IPv4 pairs.

The paper evaluates on the Graph Challenge's anonymized traffic matrices derived
from 2^30 synthetic packets (Sec. V, "Dataset"); those files are not available
here, so this module draws stand-in traffic with the same shape: Zipf-skewed
source and destination popularity over a pool of distinct 32-bit addresses,
windows of 2^10..2^17 packets, one packet per pair entry (Table I counts
packets, so every pair is one packet of weight 1).

This module only produces inputs. It holds none of the statistics' arithmetic
and is shared by the GPU path, the oracle, the tests and the benchmark. Every
random number comes from a counter-based generator (SplitMix64's finaliser
applied to a per-stream counter), so a window's packets depend only on
(config seed, stream tag, window index, packet index) and never on chunking,
thread count or device. The same functions run on numpy arrays (host) or on
torch int64 tensors (any device, used for the 2^30-packet workload); both give
bit-identical results.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
M64 = (1 << 64) - 1

# Stream tags: each random quantity draws from its own counter stream.
TAG_POOL, TAG_PERM, TAG_SRC, TAG_DST, TAG_SIZE, TAG_ARRIVAL, TAG_SCAN = 1, 2, 3, 4, 5, 6, 7


def _mix_scalar(z: int) -> int:
    """SplitMix64 output function (Steele, Lea, Flood 2014), on a Python int."""
    z &= M64
    z = ((z ^ (z >> 30)) * MIX1) & M64
    z = ((z ^ (z >> 27)) * MIX2) & M64
    return z ^ (z >> 31)


def stream_key(seed: int, tag: int, index: int = 0) -> int:
    """Derive the 64-bit key of one counter stream from (seed, tag, index)."""
    z = _mix_scalar(seed * GOLDEN + 0x1234567)
    z = _mix_scalar(z ^ (tag * 0xD1B54A32D192ED03 & M64))
    return _mix_scalar(z ^ ((index + 1) * GOLDEN & M64))


# ----------------------------------------------------------------------------
# array back ends: numpy uint64, or torch int64 (two's-complement wrap)
# ----------------------------------------------------------------------------

def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _s64(c: int) -> int:
    """A 64-bit constant as a signed int64 value."""
    c &= M64
    return c - (1 << 64) if c >> 63 else c


def _counter_u64(key: int, start: int, count: int, like=None):
    """Raw 64-bit draws number start..start+count-1 of stream `key`."""
    if like is None or not _is_torch(like):
        with np.errstate(over="ignore"):
            i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
            z = np.uint64(key) + i * np.uint64(GOLDEN)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
            return z ^ (z >> np.uint64(31))
    import torch
    dev = like.device
    i = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=dev)
    z = i * _s64(GOLDEN) + _s64(key)
    z = (z ^ ((z >> 30) & ((1 << 34) - 1))) * _s64(MIX1)
    z = (z ^ ((z >> 27) & ((1 << 37) - 1))) * _s64(MIX2)
    return z ^ ((z >> 31) & ((1 << 33) - 1))


def _uniform(raw):
    """53-bit uniform double in [0, 1) from raw 64-bit draws."""
    if _is_torch(raw):
        import torch
        return ((raw >> 11) & ((1 << 53) - 1)).to(torch.float64) * (2.0 ** -53)
    return (raw >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform(key: int, start: int, count: int, like=None):
    return _uniform(_counter_u64(key, start, count, like))


# ----------------------------------------------------------------------------
# address pool, Zipf table, rank permutation
# ----------------------------------------------------------------------------

def distinct_addresses(seed: int, count: int) -> np.ndarray:
    """`count` distinct uniform 32-bit addresses, in first-draw order."""
    key = stream_key(seed, TAG_POOL)
    got = np.empty(0, dtype=np.uint32)
    drawn = 0
    while got.size < count:
        need = count - got.size
        batch = need + need // 16 + 1024
        raw = _counter_u64(key, drawn, batch)
        drawn += batch
        cand = np.concatenate([got, (raw >> np.uint64(32)).astype(np.uint32)])
        _, first = np.unique(cand, return_index=True)
        got = cand[np.sort(first)]
    return got[:count].copy()


def zipf_cdf(n_ranks: int, s: float) -> np.ndarray:
    """Cumulative Zipf(s) probabilities over ranks 1..n_ranks (float64)."""
    w = np.arange(1, n_ranks + 1, dtype=np.float64) ** (-float(s))
    c = np.cumsum(w)
    c /= c[-1]
    c[-1] = 1.0
    return c


def rank_permutation(seed: int, n_ranks: int) -> np.ndarray:
    """Seeded permutation of 0..n_ranks-1 (destination ranks -> pool slots)."""
    raw = _counter_u64(stream_key(seed, TAG_PERM), 0, n_ranks)
    return np.argsort(raw, kind="stable").astype(np.int64)


def zipf_ranks(cdf, u):
    """0-based Zipf ranks by inverse CDF: the first rank whose CDF exceeds u."""
    if _is_torch(u):
        import torch
        r = torch.searchsorted(cdf, u, right=True)
        return torch.clamp(r, max=cdf.numel() - 1)
    r = np.searchsorted(cdf, u, side="right")
    return np.minimum(r, cdf.size - 1)


def log_uniform_sizes(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    """Window sizes floor(2^(lo + (hi-lo) u)), u uniform in [0,1)."""
    u = uniform(stream_key(seed, TAG_SIZE), 0, count)
    n = np.floor(np.exp2(lo + (hi - lo) * u)).astype(np.int64)
    return np.clip(n, 1 << lo, (1 << hi))


def poisson_arrivals(seed: int, count: int, rate: float) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    u = uniform(stream_key(seed, TAG_ARRIVAL), 0, count)
    return np.cumsum(-np.log1p(-u) / rate)


# ----------------------------------------------------------------------------
# workload description and window generation
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    seed: int
    pool_size: int
    s_src: float
    s_dst: float
    sizes: np.ndarray                      # packets per window (int64)
    scan_frac: float = 0.0                 # fraction of packets from scanner / to sink
    scan_targets: int = 1 << 16
    arrivals: np.ndarray | None = None     # arrival times for serving (s)
    _pool: np.ndarray | None = field(default=None, repr=False)
    _perm: np.ndarray | None = field(default=None, repr=False)
    _cdf_src: np.ndarray | None = field(default=None, repr=False)
    _cdf_dst: np.ndarray | None = field(default=None, repr=False)

    @property
    def num_windows(self) -> int:
        return int(self.sizes.size)

    @property
    def offsets(self) -> np.ndarray:
        off = np.zeros(self.num_windows + 1, dtype=np.int64)
        np.cumsum(self.sizes, out=off[1:])
        return off

    @property
    def total_packets(self) -> int:
        return int(self.sizes.sum())

    def _setup(self):
        if self._pool is not None:
            return
        extra = 2 + 2 * self.scan_targets if self.scan_frac > 0 else 0
        addrs = distinct_addresses(self.seed, self.pool_size + extra)
        self._pool = addrs[: self.pool_size]
        if extra:
            rest = addrs[self.pool_size:]
            self.scanner, self.sink = int(rest[0]), int(rest[1])
            self.targets = rest[2: 2 + self.scan_targets]
            self.sources = rest[2 + self.scan_targets:]
        self._perm = rank_permutation(self.seed, self.pool_size)
        self._cdf_src = zipf_cdf(self.pool_size, self.s_src)
        self._cdf_dst = zipf_cdf(self.pool_size, self.s_dst)

    def scan_count(self, n: int) -> int:
        return int(math.floor(self.scan_frac * n + 0.5)) if self.scan_frac > 0 else 0

    def window(self, w: int, device=None):
        """(src, dst) uint32 arrays of window w (numpy), or int32 torch tensors
        holding the same bits when `device` is given."""
        self._setup()
        n = int(self.sizes[w])
        if device is None:
            return self._window_np(w, n)
        return self._window_torch(w, n, device)

    def _window_np(self, w: int, n: int):
        us = uniform(stream_key(self.seed, TAG_SRC, w), 0, n)
        ud = uniform(stream_key(self.seed, TAG_DST, w), 0, n)
        src = self._pool[zipf_ranks(self._cdf_src, us)]
        dst = self._pool[self._perm[zipf_ranks(self._cdf_dst, ud)]]
        m = self.scan_count(n)
        if m:
            pos, j = self._scan_positions(w, n, m)
            src[pos[:m]] = self.scanner
            dst[pos[:m]] = self.targets[(w * m + j) % self.scan_targets]
            src[pos[m:]] = self.sources[(w * m + j) % self.scan_targets]
            dst[pos[m:]] = self.sink
        return src, dst

    def _window_torch(self, w: int, n: int, device):
        import torch
        like = torch.empty(0, device=device)
        cache = getattr(self, "_tcache", None)
        if cache is None or cache[0] != str(device):
            pool = torch.from_numpy(self._pool.astype(np.int64)).to(device)
            cache = (str(device), pool,
                     torch.from_numpy(self._perm).to(device),
                     torch.from_numpy(self._cdf_src).to(device),
                     torch.from_numpy(self._cdf_dst).to(device))
            self._tcache = cache
        _, pool, perm, cs, cd = cache
        us = uniform(stream_key(self.seed, TAG_SRC, w), 0, n, like)
        ud = uniform(stream_key(self.seed, TAG_DST, w), 0, n, like)
        src = pool[zipf_ranks(cs, us)]
        dst = pool[perm[zipf_ranks(cd, ud)]]
        m = self.scan_count(n)
        if m:
            pos, j = self._scan_positions(w, n, m)
            pos_t = torch.from_numpy(pos).to(device)
            jj = (w * m + j) % self.scan_targets
            tg = torch.from_numpy(self.targets[jj].astype(np.int64)).to(device)
            sc = torch.from_numpy(self.sources[jj].astype(np.int64)).to(device)
            src[pos_t[:m]] = self.scanner
            dst[pos_t[:m]] = tg
            src[pos_t[m:]] = sc
            dst[pos_t[m:]] = self.sink
        # reinterpret the low 32 bits as int32 (same bits as uint32)
        return (_to_i32(src), _to_i32(dst))

    def _scan_positions(self, w: int, n: int, m: int):
        """2m distinct positions (a + k*b) mod n, b coprime to n: the first m
        carry scanner packets, the next m sink packets."""
        raw = _counter_u64(stream_key(self.seed, TAG_SCAN, w), 0, 2)
        a = int(raw[0]) % n
        b = (int(raw[1]) % n) | 1
        while math.gcd(b, n) != 1:
            b += 2
        k = np.arange(2 * m, dtype=np.int64)
        pos = (a + k * b) % n
        return pos, np.arange(m, dtype=np.int64)

    def concat(self, windows=None):
        """Concatenated (src, dst) numpy arrays of the given windows (default all)."""
        ws = range(self.num_windows) if windows is None else windows
        parts = [self.window(w) for w in ws]
        if not parts:
            return np.empty(0, np.uint32), np.empty(0, np.uint32)
        return (np.concatenate([p[0] for p in parts]),
                np.concatenate([p[1] for p in parts]))

    def device_concat(self, device, windows=None):
        """Concatenated int32 tensors (uint32 bits) on `device`, built window by window."""
        import torch
        ws = list(range(self.num_windows)) if windows is None else list(windows)
        total = int(sum(int(self.sizes[w]) for w in ws))
        src = torch.empty(total, dtype=torch.int32, device=device)
        dst = torch.empty(total, dtype=torch.int32, device=device)
        o = 0
        for w in ws:
            s, d = self.window(w, device=device)
            src[o:o + s.numel()] = s
            dst[o:o + d.numel()] = d
            o += s.numel()
        return src, dst


def _to_i32(x):
    import torch
    x = x & 0xFFFFFFFF
    return torch.where(x >= (1 << 31), x - (1 << 32), x).to(torch.int32)


def as_u32(t) -> np.ndarray:
    """Host uint32 view of a torch int32 tensor (bit reinterpretation)."""
    return t.detach().cpu().numpy().view(np.uint32)


# ----------------------------------------------------------------------------
# the five workloads (seed = workload number)
# ----------------------------------------------------------------------------

def one_window(n: int = 1 << 17) -> Workload:
    """One window of 2^17 packets, Zipf(1.2) sources and destinations over a pool of 2^16."""
    return Workload("one_window_2^17", 1, 1 << 16, 1.2, 1.2, np.array([n], np.int64))


def windows64(num: int = 64, n: int = 1 << 17) -> Workload:
    """64 windows of 2^17 packets; sources Zipf(1.1), destinations Zipf(1.3), pool 2^20."""
    return Workload("64x2^17_plus_aggregate", 2, 1 << 20, 1.1, 1.3,
                    np.full(num, n, np.int64))


def uneven1024(num: int = 1024, lo: int = 12, hi: int = 17) -> Workload:
    """1024 windows, sizes log-uniform in 2^12..2^17, Zipf(1.2) over a pool of 2^22."""
    return Workload("1024_uneven_2^12..2^17", 3, 1 << 22, 1.2, 1.2,
                    log_uniform_sizes(3, num, lo, hi))


def aggregate_2p30(num: int = 8192, n: int = 1 << 17) -> Workload:
    """8192 windows of 2^17 (2^30 packets), Zipf(1.2) over 2^22, with 1% of each
    window's packets from one scanner to 2^16 targets and 1% to one sink from
    2^16 sources."""
    return Workload("aggregate_2^30_scanner_sink", 4, 1 << 22, 1.2, 1.2,
                    np.full(num, n, np.int64), scan_frac=0.01)


def serving(num: int = 11264, lo: int = 10, hi: int = 17, rate: float = 2000.0) -> Workload:
    """Serving: window sizes log-uniform 2^10..2^17, Zipf(1.2) over 2^22, Poisson arrivals."""
    wl = Workload("serving_poisson_2000/s", 5, 1 << 22, 1.2, 1.2,
                  log_uniform_sizes(5, num, lo, hi))
    wl.arrivals = poisson_arrivals(5, num, rate)
    return wl


WORKLOADS = {
    "one_window": one_window,
    "windows64": windows64,
    "uneven1024": uneven1024,
    "aggregate_2p30": aggregate_2p30,
    "serving": serving,
}
