"""Thin ctypes binding of libns.so (include/ns.h).

Argument marshalling only: torch tensors supply device memory, the current
torch stream supplies the HIP stream, and every step of the computation runs in
the library's HIP kernels. There is no CPU fallback: if libns.so is missing or
no GPU is present, calls raise.

Bit conventions: addresses travel as int32 tensors holding uint32 bits; keys
and counts as int64 tensors holding uint64 bits.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libns.so")
# the same library with every scatter / gather index of the radix passes and
# run scans checked against its bound (a violation raises NS_ERR_BOUNDS)
DEBUG_LIB_PATH = os.path.join(HERE, "libns_debug.so")

STAT_NAMES = (
    "valid_packets", "unique_links", "unique_sources", "unique_destinations",
    "max_source_packets", "max_source_fanout", "max_destination_packets",
    "max_destination_fanin",
)

NS_OK = 0
ERRORS = {
    -1: "NS_ERR_INVALID_ARG", -2: "NS_ERR_CAPACITY", -3: "NS_ERR_WORKSPACE",
    -4: "NS_ERR_HIP", -5: "NS_ERR_UNDERFLOW", -6: "NS_ERR_UNSUPPORTED", -7: "NS_ERR_BOUNDS",
}


class NSError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({_lib_error_string(code)})")


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in STAT_NAMES]


class MatrixView(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("counts", ctypes.c_void_p), ("nnz", ctypes.c_void_p),
                ("capacity", ctypes.c_uint64), ("packets", ctypes.c_uint64)]


class Tuning(ctypes.Structure):
    _fields_ = [("sort_block", ctypes.c_uint32), ("sort_items", ctypes.c_uint32),
                ("digit_bits", ctypes.c_uint32), ("scan_items", ctypes.c_uint32),
                ("chunked_min", ctypes.c_uint64)]


class RollingView(ctypes.Structure):
    _fields_ = [("mem", ctypes.c_void_p), ("bytes", ctypes.c_uint64),
                ("link_slots", ctypes.c_uint64), ("address_slots", ctypes.c_uint64)]


class BatchMatricesView(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("counts", ctypes.c_void_p),
                ("nnz", ctypes.c_void_p), ("capacity", ctypes.c_uint64)]


EXPORTS = ("ns_workspace_size", "ns_build_matrix", "ns_accumulate_workspace_size",
           "ns_accumulate", "ns_accumulate_noalloc", "ns_stats",
           "ns_stream_workspace_size", "ns_build_matrix_streamed",
           "ns_stats_csr_workspace_size", "ns_stats_csr",
           "ns_batch_stats", "ns_batch_stats_eager", "ns_max_link_packets",
           "ns_batch_max_link_packets", "ns_rolling_size", "ns_rolling_init",
           "ns_rolling_update", "ns_rolling_compact", "ns_rolling_occupancy",
           "ns_device_status", "ns_release_graphs",
           "ns_timing_enable", "ns_timing_reset", "ns_timing_read",
           "ns_error_string", "ns_version")

# kernel kinds of ns_timing_read
KINDS = ("fill", "tiles", "hist", "hist_scan", "pass0", "pass", "col_pass", "rle", "runs",
         "segmax", "finalize", "merge", "chunk_count", "pass0_chunked", "pass_chunked",
         "col_pass_chunked", "small")
# default single-segment size from which sorts use the chunked passes
# (ns_tuning_t.chunked_min = 0)
CHUNKED_MIN_DEFAULT = 1 << 24
# launch shape (workgroup size, keys per thread) of the chunked passes
CHUNKED_SHAPE = (512, 16)

_lib = None


def load(path: str = LIB_PATH):
    """Load libns.so and declare its signatures (no GPU needed to load)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libns.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P, U64, U32, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    PM = ctypes.POINTER(MatrixView)
    lib.ns_workspace_size.argtypes = [U64, U32, ctypes.POINTER(U64)]
    lib.ns_build_matrix.argtypes = [P, P, U64, PM, P, U64, P]
    lib.ns_accumulate.argtypes = [PM, PM, I, PM, P, U64, P]
    lib.ns_accumulate_noalloc.argtypes = [PM, PM, I, PM, P]
    lib.ns_stream_workspace_size.argtypes = [U64, U64, ctypes.POINTER(U64)]
    lib.ns_accumulate_workspace_size.argtypes = [U64, U64, ctypes.POINTER(U64)]
    lib.ns_stats_csr_workspace_size.argtypes = [U64, ctypes.POINTER(U64)]
    lib.ns_stats_csr.argtypes = [P, P, U64, P, P, U64, U64, P, P, U64, P]
    lib.ns_build_matrix_streamed.argtypes = [P, P, U64, U64, PM, P, U64, P, P]
    lib.ns_stats.argtypes = [PM, P, P, U64, P]
    batch = [P, P, P, U32, U64, P, PM, P, ctypes.POINTER(BatchMatricesView),
             ctypes.POINTER(Tuning), P, U64, P]
    lib.ns_batch_stats.argtypes = batch
    lib.ns_batch_stats_eager.argtypes = batch
    lib.ns_max_link_packets.argtypes = [PM, P, P]
    lib.ns_batch_max_link_packets.argtypes = [ctypes.POINTER(BatchMatricesView), P, U32, U64, P, P]
    PR = ctypes.POINTER(RollingView)
    lib.ns_rolling_size.argtypes = [U64, U64, ctypes.POINTER(U64)]
    lib.ns_rolling_init.argtypes = [PR, P]
    lib.ns_rolling_update.argtypes = [PR, PM, PM, P, P]
    lib.ns_rolling_compact.argtypes = [PR, PR, P]
    lib.ns_rolling_occupancy.argtypes = [PR, P, P]
    lib.ns_device_status.argtypes = [P, ctypes.POINTER(I)]
    lib.ns_release_graphs.argtypes = []
    lib.ns_timing_enable.argtypes = [I]
    lib.ns_timing_reset.argtypes = []
    lib.ns_timing_read.argtypes = [U32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(U64)]
    lib.ns_error_string.argtypes = [I]
    lib.ns_error_string.restype = ctypes.c_char_p
    lib.ns_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("ns_error_string", "ns_version"):
            getattr(lib, name).restype = I
    _lib = lib
    return lib


def _lib_error_string(code: int) -> str:
    try:
        return load().ns_error_string(code).decode()
    except Exception:  # the message is best effort
        return "?"


def _check(rc: int, where: str):
    if rc != NS_OK:
        raise NSError(rc, where)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libns needs a ROCm GPU; none is visible")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() else 0)


def workspace_size(max_packets: int, num_windows: int = 1) -> int:
    out = ctypes.c_uint64()
    _check(load().ns_workspace_size(max_packets, num_windows, ctypes.byref(out)),
           "ns_workspace_size")
    return int(out.value)


class Workspace:
    """Caller-owned scratch memory for the library (a torch uint8 buffer)."""

    def __init__(self, max_packets: int, num_windows: int = 1, device="cuda"):
        torch = _torch()
        self.max_packets, self.num_windows = int(max_packets), int(num_windows)
        self.nbytes = workspace_size(self.max_packets, self.num_windows)
        self.buf = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        assert self.buf.data_ptr() % 256 == 0

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())


class Matrix:
    """Device traffic matrix in sorted COO form (keys, counts, nnz) + packets."""

    def __init__(self, capacity: int, device="cuda"):
        torch = _torch()
        self.capacity = int(capacity)
        n = max(self.capacity, 1)
        self.keys = torch.empty(n, dtype=torch.int64, device=device)
        self.counts = torch.empty(n, dtype=torch.int64, device=device)
        self.nnz_t = torch.zeros(1, dtype=torch.int64, device=device)
        self.packets = 0

    @classmethod
    def wrap(cls, keys, counts, nnz_t, capacity: int, packets: int) -> "Matrix":
        """A Matrix over existing device tensors (no allocation)."""
        m = cls.__new__(cls)
        m.keys, m.counts, m.nnz_t = keys, counts, nnz_t
        m.capacity, m.packets = int(capacity), int(packets)
        return m

    def view(self) -> MatrixView:
        return MatrixView(self.keys.data_ptr(), self.counts.data_ptr(), self.nnz_t.data_ptr(),
                          self.capacity, self.packets)

    def nnz(self) -> int:
        return int(self.nnz_t.item())

    def numpy(self):
        """Host copies (uint64) of the first nnz keys and counts."""
        n = self.nnz()
        k = self.keys[:n].cpu().numpy().view(np.uint64)
        c = self.counts[:n].cpu().numpy().view(np.uint64)
        return k, c


def _u32_tensor(x):
    torch = _torch()
    assert x.dtype == torch.int32 and x.is_cuda and x.is_contiguous(), "int32 cuda contiguous"
    return x


def build_matrix(src, dst, out: Matrix, ws: Workspace, stream=None) -> Matrix:
    """ns_build_matrix: traffic matrix of one window."""
    _u32_tensor(src), _u32_tensor(dst)
    n = src.numel()
    assert dst.numel() == n
    v = out.view()
    _check(load().ns_build_matrix(_ptr(src), _ptr(dst), n, ctypes.byref(v), ws.ptr, ws.nbytes,
                                  _stream(stream)), "ns_build_matrix")
    out.packets = int(v.packets)
    return out


def stream_workspace_size(batch: int, capacity: int) -> int:
    out = ctypes.c_uint64()
    _check(load().ns_stream_workspace_size(int(batch), int(capacity), ctypes.byref(out)),
           "ns_stream_workspace_size")
    return int(out.value)


class StreamWorkspace:
    """Device scratch memory of ns_build_matrix_streamed for sub-partitions of
    `batch` packets and an aggregate of `capacity` links."""

    def __init__(self, batch: int, capacity: int, device="cuda"):
        torch = _torch()
        self.batch, self.capacity = int(batch), int(capacity)
        self.nbytes = stream_workspace_size(self.batch, self.capacity)
        self.buf = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        assert self.buf.data_ptr() % 256 == 0

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())


def build_matrix_streamed(src, dst, out: Matrix, ws: StreamWorkspace, stream=None,
                          copy_stream=None) -> Matrix:
    """ns_build_matrix_streamed: the matrix of host-resident packets (int32 CPU
    tensors in page-locked memory, e.g. torch.empty(..., pin_memory=True)),
    built in sub-partitions of ws.batch packets. Pageable tensors are refused
    (the library would reject them too)."""
    torch = _torch()
    for x in (src, dst):
        assert x.dtype == torch.int32 and not x.is_cuda and x.is_contiguous(), \
            "int32 host contiguous"
        if x.numel() and not x.is_pinned():
            raise ValueError("ns_build_matrix_streamed needs page-locked host memory "
                             "(pin_memory=True)")
    n = src.numel()
    assert dst.numel() == n
    v = out.view()
    cs = ctypes.c_void_p(copy_stream.cuda_stream) if copy_stream is not None else ctypes.c_void_p(0)
    _check(load().ns_build_matrix_streamed(_ptr(src), _ptr(dst), n, ws.batch, ctypes.byref(v),
                                           ws.ptr, ws.nbytes, _stream(stream), cs),
           "ns_build_matrix_streamed")
    out.packets = int(v.packets)
    return out


def accumulate_workspace_size(na: int, nb: int) -> int:
    out = ctypes.c_uint64()
    _check(load().ns_accumulate_workspace_size(int(na), int(nb), ctypes.byref(out)),
           "ns_accumulate_workspace_size")
    return int(out.value)


class MergeWorkspace:
    """Device scratch memory of ns_accumulate for inputs of at most `na` and
    `nb` entries (far smaller than a Workspace, which also serves)."""

    def __init__(self, na: int, nb: int, device="cuda"):
        torch = _torch()
        self.nbytes = accumulate_workspace_size(na, nb)
        self.buf = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        assert self.buf.data_ptr() % 256 == 0

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())


def accumulate(acc_in: Matrix, win: Matrix, sign: int, acc_out: Matrix,
               ws: "Workspace | MergeWorkspace", stream=None) -> Matrix:
    """ns_accumulate: acc_out = acc_in + sign * win (union-add / subtract)."""
    a, b, c = acc_in.view(), win.view(), acc_out.view()
    _check(load().ns_accumulate(ctypes.byref(a), ctypes.byref(b), int(sign), ctypes.byref(c),
                                ws.ptr, ws.nbytes, _stream(stream)), "ns_accumulate")
    acc_out.packets = int(c.packets)
    return acc_out


def accumulate_noalloc(acc_in: Matrix, win: Matrix, sign: int, acc_out: Matrix, stream=None):
    """ns_accumulate_noalloc: the same union-add / subtract as accumulate(),
    with the library's own device scratch instead of a caller workspace (no
    device memory is allocated; calls that overlap on one device race)."""
    a, b, c = acc_in.view(), win.view(), acc_out.view()
    _check(load().ns_accumulate_noalloc(ctypes.byref(a), ctypes.byref(b), int(sign),
                                        ctypes.byref(c), _stream(stream)),
           "ns_accumulate_noalloc")
    acc_out.packets = int(c.packets)
    return acc_out


# largest na + nb that ns_accumulate_noalloc accepts (NS_ACCUMULATE_NOALLOC_MAX_ENTRIES)
ACCUMULATE_NOALLOC_MAX_ENTRIES = 1 << 30


def stats(m: Matrix, out, ws: Workspace, stream=None):
    """ns_stats into `out` (int64 cuda tensor of 8)."""
    v = m.view()
    assert out.numel() >= 8 and out.dtype.itemsize == 8
    _check(load().ns_stats(ctypes.byref(v), _ptr(out), ws.ptr, ws.nbytes, _stream(stream)),
           "ns_stats")
    return out


def stats_csr_workspace_size(nnz: int) -> int:
    out = ctypes.c_uint64()
    _check(load().ns_stats_csr_workspace_size(int(nnz), ctypes.byref(out)),
           "ns_stats_csr_workspace_size")
    return int(out.value)


def stats_csr(rows, row_ptr, cols, vals, packets: int, out, ws=None, stream=None):
    """ns_stats_csr: the eight quantities of a hypersparse CSR matrix (device
    tensors: rows int32 [nrows] source addresses, row_ptr int64 [nrows+1],
    cols int32 [nnz] destination addresses, vals int64 [nnz]) into `out`
    (int64 cuda tensor of 8). `ws`: a uint8 cuda tensor of at least
    stats_csr_workspace_size(nnz) bytes (allocated here when None)."""
    torch = _torch()
    nnz, nrows = cols.numel(), rows.numel()
    assert vals.numel() == nnz and row_ptr.numel() == nrows + 1
    need = stats_csr_workspace_size(nnz)
    if ws is None:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=cols.device)
    assert ws.numel() >= need and ws.data_ptr() % 256 == 0
    _check(load().ns_stats_csr(_ptr(rows), _ptr(row_ptr), nrows, _ptr(cols), _ptr(vals), nnz,
                               int(packets), _ptr(out), ctypes.c_void_p(ws.data_ptr()),
                               ws.numel(), _stream(stream)), "ns_stats_csr")
    return out


class BatchMatrices:
    """Per-window matrices of a batch, laid out by packet offset: window w's
    entries start at the window's first packet position; nnz[w] on the device."""

    def __init__(self, capacity: int, num_windows: int, device="cuda", keys=None, counts=None):
        torch = _torch()
        self.capacity = int(capacity)
        n = max(self.capacity, 1)
        self.keys = keys if keys is not None else torch.empty(n, dtype=torch.int64, device=device)
        self.counts = counts if counts is not None else torch.empty(n, dtype=torch.int64,
                                                                     device=device)
        self.nnz = torch.zeros(max(num_windows, 1), dtype=torch.int64, device=device)

    def view(self) -> BatchMatricesView:
        return BatchMatricesView(self.keys.data_ptr(), self.counts.data_ptr(),
                                 self.nnz.data_ptr(), self.capacity)

    def window(self, w: int, start: int, n: int) -> "Matrix":
        """Matrix view of window w, whose packets were [start, start + n) of the batch."""
        return Matrix.wrap(self.keys[start:start + max(n, 1)],
                           self.counts[start:start + max(n, 1)], self.nnz[w:w + 1], n, n)


def tuning(sort_block=0, sort_items=0, digit_bits=0, scan_items=0, chunked_min=0) -> Tuning:
    return Tuning(sort_block, sort_items, digit_bits, scan_items, chunked_min)


def max_link_packets(m: Matrix, out, stream=None):
    """ns_max_link_packets into `out` (int64 cuda tensor, first element)."""
    v = m.view()
    assert out.numel() >= 1 and out.dtype.itemsize == 8 and out.is_cuda
    _check(load().ns_max_link_packets(ctypes.byref(v), _ptr(out), _stream(stream)),
           "ns_max_link_packets")
    return out


def batch_max_link_packets(win: "BatchMatrices", offsets, out, stream=None):
    """ns_batch_max_link_packets: out[w] (int64 cuda [W]) = largest link count of
    window w's matrix in `win` (written by batch_stats with these offsets)."""
    torch = _torch()
    assert offsets.dtype == torch.int64 and offsets.is_cuda
    W = offsets.numel() - 1
    assert out.numel() >= W and out.dtype.itemsize == 8 and out.is_cuda
    wv = win.view()
    N = int(win.capacity)
    _check(load().ns_batch_max_link_packets(ctypes.byref(wv), _ptr(offsets), W, N, _ptr(out),
                                            _stream(stream)), "ns_batch_max_link_packets")
    return out


def batch_stats(src, dst, offsets, out, ws: Workspace, agg: Matrix | None = None,
                agg_stats=None, win: BatchMatrices | None = None, tune: Tuning | None = None,
                stream=None, graph: bool = True):
    """ns_batch_stats (graph=True) or ns_batch_stats_eager: per-window stats
    into out (int64 cuda [W, 8]); optionally the aggregate matrix and its stats,
    and each window's own matrix. out=None with an aggregate computes the
    aggregate alone."""
    torch = _torch()
    _u32_tensor(src), _u32_tensor(dst)
    assert offsets.dtype == torch.int64 and offsets.is_cuda
    W = offsets.numel() - 1
    N = src.numel()
    assert out is None or out.numel() >= 8 * W
    av = agg.view() if agg is not None else None
    wv = win.view() if win is not None else None
    fn = load().ns_batch_stats if graph else load().ns_batch_stats_eager
    rc = fn(_ptr(src), _ptr(dst), _ptr(offsets), W, N, _ptr(out) if out is not None else None,
            ctypes.byref(av) if av is not None else None,
            _ptr(agg_stats) if agg_stats is not None else None,
            ctypes.byref(wv) if wv is not None else None,
            ctypes.byref(tune) if tune is not None else None,
            ws.ptr, ws.nbytes, _stream(stream))
    _check(rc, "ns_batch_stats")
    if agg is not None:
        agg.packets = int(av.packets)
    return out


class RollingState:
    """Device hash-table state of a rolling aggregate (ns_rolling_*)."""

    def __init__(self, link_slots: int = 1 << 25, address_slots: int = 1 << 23, device="cuda",
                 stream=None):
        torch = _torch()
        out = ctypes.c_uint64()
        _check(load().ns_rolling_size(link_slots, address_slots, ctypes.byref(out)),
               "ns_rolling_size")
        self.nbytes = int(out.value)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.link_slots, self.address_slots = int(link_slots), int(address_slots)
        self.clear(stream)

    def view(self) -> RollingView:
        return RollingView(self.buf.data_ptr(), self.nbytes, self.link_slots, self.address_slots)

    def clear(self, stream=None):
        v = self.view()
        _check(load().ns_rolling_init(ctypes.byref(v), _stream(stream)), "ns_rolling_init")


def rolling_update(state: RollingState, add: Matrix | None, remove: Matrix | None, out,
                   stream=None):
    """A <- A + add - remove on the rolling state; the eight quantities of A into out."""
    r = state.view()
    a = add.view() if add is not None else None
    b = remove.view() if remove is not None else None
    _check(load().ns_rolling_update(ctypes.byref(r), ctypes.byref(a) if a is not None else None,
                                    ctypes.byref(b) if b is not None else None, _ptr(out),
                                    _stream(stream)), "ns_rolling_update")
    return out


def rolling_compact(src: RollingState, dst: RollingState, stream=None):
    a, b = src.view(), dst.view()
    _check(load().ns_rolling_compact(ctypes.byref(a), ctypes.byref(b), _stream(stream)),
           "ns_rolling_compact")


def rolling_occupancy(state: RollingState, out, stream=None):
    """Slots taken in the link, source and destination tables since the last
    clear or compaction, into out (3 int64, device)."""
    v = state.view()
    _check(load().ns_rolling_occupancy(ctypes.byref(v), _ptr(out), _stream(stream)),
           "ns_rolling_occupancy")
    return out


def device_status(stream=None) -> int:
    st = ctypes.c_int()
    _check(load().ns_device_status(_stream(stream), ctypes.byref(st)), "ns_device_status")
    return int(st.value)


def timing_enable(on: bool = True):
    _check(load().ns_timing_enable(1 if on else 0), "ns_timing_enable")


def timing_reset():
    _check(load().ns_timing_reset(), "ns_timing_reset")


def timing_read() -> dict:
    """{kind: (total_ms, launches)} for every kernel kind seen since the last reset."""
    out = {}
    for i, name in enumerate(KINDS):
        ms, n = ctypes.c_double(), ctypes.c_uint64()
        _check(load().ns_timing_read(i, ctypes.byref(ms), ctypes.byref(n)), "ns_timing_read")
        if n.value:
            out[name] = (float(ms.value), int(n.value))
    return out


def release_graphs():
    _check(load().ns_release_graphs(), "ns_release_graphs")


def version() -> str:
    return load().ns_version().decode()


def stats_numpy(t) -> np.ndarray:
    """uint64 host view of a stats tensor ([8] or [W, 8])."""
    return t.detach().cpu().numpy().view(np.uint64)
