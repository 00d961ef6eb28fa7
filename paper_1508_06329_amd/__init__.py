"""LexBFS chordality test on MI355X (gfx950).

Python binding of ``liblexbfs.so`` (C ABI in ``include/lexbfs.h``). PyTorch
supplies device memory and streams; every step of the path runs in the HIP
kernels: the LexBFS order (Section 6.1 of Lupinska, "A Parallel Algorithm to
Test Chordality of Graphs"), the perfect-elimination test (Section 6.2), and
a chordless-cycle certificate for non-chordal graphs. Multi-sweep LexBFS
(LexBFS+) and the three-sweep unit interval test build on the same LexBFS
kernel (the interval direction of Sections 3.2 and 8).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import (LEXBFS_FLAG_FORCE_FALLBACK, LEXBFS_FLAG_MCS, LEXBFS_FLAG_PER_STEP, LEXBFS_FLAG_VALIDATE, LEXBFS_MAX_N,
                   LexbfsError, lexbfs_graph_t, lexbfs_outputs_t, lexbfs_result_t, lexbfs_tuning_t)

__all__ = ["BatchPlan", "pack_graphs", "build_bitset", "KernelTimer", "DeviceGraph", "Result", "lexbfs_order", "chordal_test", "chordal_test_batch", "workspace_bytes",
           "lexbfs_plus", "unit_interval_test", "unit_interval_test_batch", "IntervalResult",
           "batch_workspace_bytes", "LexbfsError", "LEXBFS_MAX_N", "LEXBFS_FLAG_FORCE_FALLBACK",
           "LEXBFS_FLAG_PER_STEP", "LEXBFS_FLAG_MCS", "LEXBFS_FLAG_VALIDATE", "validate"]


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> Optional[int]:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _on_stream(stream: Optional[torch.cuda.Stream], *tensors: Optional[torch.Tensor]) -> None:
    """Tensors allocated on the current stream but used by kernels on
    another one: tell the caching allocator, so that freeing them (a
    temporary workspace dropped on return, an output the caller drops) does
    not hand their memory to a new allocation while those kernels run."""
    if stream is None or stream == torch.cuda.current_stream(stream.device):
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def _zeros_on(shape, device, stream: Optional[torch.cuda.Stream]) -> torch.Tensor:
    """A zero-filled int32 device tensor whose fill runs on `stream` (the
    current stream if None): ahead of the kernels later queued there, which
    a fill on another stream would not be."""
    if stream is None:
        return torch.zeros(shape, dtype=torch.int32, device=device)
    with torch.cuda.stream(stream):
        return torch.zeros(shape, dtype=torch.int32, device=device)


def _wait(stream: Optional[torch.cuda.Stream]) -> None:
    (stream if stream is not None else torch.cuda.current_stream()).synchronize()


class DeviceGraph:
    """A graph resident in device memory: int32 CSR plus the n x W uint64
    adjacency bitset (stored in an int64 tensor of the same bits)."""

    def __init__(self, n: int, W: int, row_ptr: torch.Tensor, col_idx: torch.Tensor, bits: torch.Tensor):
        self.n, self.W = int(n), int(W)
        self.row_ptr, self.col_idx, self.bits = row_ptr, col_idx, bits
        self.nnz = int(col_idx.numel()) if n > 0 else 0

    @classmethod
    def from_host(cls, g, device="cuda") -> "DeviceGraph":
        """From an object with n, W, row_ptr, col_idx, bits numpy arrays."""
        rp = torch.from_numpy(g.row_ptr).to(device)
        ci = torch.from_numpy(g.col_idx if g.col_idx.size else g.col_idx.reshape(0)).to(device)
        if ci.numel() == 0:
            ci = torch.zeros(1, dtype=torch.int32, device=device)[:0]
        bits = torch.from_numpy(g.bits.view("int64")).to(device)
        return cls(g.n, g.W, rp, ci, bits)

    @classmethod
    def from_host_csr(cls, g, device="cuda", stream=None) -> "DeviceGraph":
        """From a host CSR only (an object with n, row_ptr and col_idx numpy
        arrays): the CSR is staged in pinned host memory and copied
        asynchronously on `stream` (the current stream if None), then the
        bitset is built on the device there (lexbfs_build_bitset). Only the
        CSR crosses PCIe, and the call returns without waiting; work queued
        on the same stream afterwards sees the finished graph."""
        import numpy as np

        dev = torch.device(device)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        n = int(g.n)
        nnz = int(g.row_ptr[n]) if n > 0 else 0
        rp_h = torch.from_numpy(np.ascontiguousarray(g.row_ptr[: n + 1], dtype=np.int32)).pin_memory()
        ci_h = torch.from_numpy(np.ascontiguousarray(g.col_idx[:nnz], dtype=np.int32)).pin_memory()
        with torch.cuda.stream(s):
            rp = torch.empty(rp_h.numel(), dtype=torch.int32, device=dev)
            ci = torch.empty(nnz, dtype=torch.int32, device=dev)
            rp.copy_(rp_h, non_blocking=True)
            if nnz:
                ci.copy_(ci_h, non_blocking=True)
        return cls.from_csr(n, rp, ci, stream=s)

    @classmethod
    def from_csr(cls, n: int, row_ptr: torch.Tensor, col_idx: torch.Tensor, words_per_row: Optional[int] = None,
                 stream=None) -> "DeviceGraph":
        """From a device-resident CSR: the bitset is built on the device
        (lexbfs_build_bitset), so only the CSR has to cross PCIe."""
        W = int(words_per_row) if words_per_row is not None else (n + 63) // 64
        bits = build_bitset(n, row_ptr, col_idx, W, stream)
        return cls(n, W, row_ptr, col_idx, bits)

    def desc(self) -> lexbfs_graph_t:
        d = lexbfs_graph_t()
        d.n = self.n
        d.reserved = 0
        d.nnz = self.nnz
        d.row_ptr = self.row_ptr.data_ptr() if self.n > 0 else None
        d.col_idx = self.col_idx.data_ptr() if self.nnz > 0 else None
        d.bits = self.bits.data_ptr() if self.n > 0 else None
        d.words_per_row = self.W
        return d

    @property
    def device(self):
        return self.row_ptr.device


@dataclass
class Result:
    chordal: bool
    witness: tuple
    cycle_len: int
    fallback: bool
    order: Optional[torch.Tensor] = None
    rank: Optional[torch.Tensor] = None
    parent: Optional[torch.Tensor] = None
    cycle: Optional[torch.Tensor] = None

    @property
    def cycle_list(self) -> List[int]:
        if self.cycle is None or self.cycle_len == 0:
            return []
        return self.cycle[: self.cycle_len].tolist()

    @classmethod
    def from_record(cls, row: torch.Tensor, **outputs) -> "Result":
        """Decode a result record (8 int32) that the library wrote."""
        chordal, wit, clen, fb = _result_from(row.cpu())
        return cls(chordal, wit, clen, fb, **outputs)


class KernelTimer:
    """HIP-event timing of every library kernel launch while active.

    with KernelTimer() as kt: ...; kt.result() -> {kind: (launches, total_ms)}
    """

    def __enter__(self):
        _lib.check(_lib.load().lexbfs_profile_enable(1), "lexbfs_profile_enable")
        self.collect()  # discard anything older
        return self

    def collect(self):
        lib = _lib.load()
        counts = (ctypes.c_int32 * _lib.LEXBFS_KERNEL_KINDS)()
        ms = (ctypes.c_double * _lib.LEXBFS_KERNEL_KINDS)()
        rc = lib.lexbfs_profile_collect(counts, ms)
        if rc < 0:
            _lib.check(rc, "lexbfs_profile_collect")
        self.dropped = rc
        self.last = {name: (int(counts[i]), float(ms[i])) for i, name in enumerate(_lib.KERNEL_KIND_NAMES)}
        return self.last

    def __exit__(self, *exc):
        _lib.load().lexbfs_profile_enable(0)
        return False


def build_bitset(n: int, row_ptr: torch.Tensor, col_idx: torch.Tensor, words_per_row: Optional[int] = None,
                 stream=None) -> torch.Tensor:
    """The n x words_per_row packed adjacency bitset (int64 tensor holding
    the uint64 words) built on the device from a device CSR."""
    W = int(words_per_row) if words_per_row is not None else (n + 63) // 64
    bits = torch.empty(max(n * W, 1), dtype=torch.int64, device=row_ptr.device)
    if n > 0:
        rc = _lib.load().lexbfs_build_bitset(n, row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None,
                                             bits.data_ptr(), W, _stream_handle(stream))
        _lib.check(rc, "lexbfs_build_bitset")
        _on_stream(stream, bits)
    return bits


def validate(g: DeviceGraph, stream=None) -> None:
    """Check the input contract on the device (lexbfs_validate); raises
    LexbfsError with code LEXBFS_EGRAPH (-4) naming the broken rule."""
    ws = _workspace(256, g.device)
    rc = _lib.load().lexbfs_validate(ctypes.byref(g.desc()), ws.data_ptr(), ws.numel(), _stream_handle(stream))
    _lib.check(rc, "lexbfs_validate")


def workspace_bytes(n: int) -> int:
    return int(_lib.load().lexbfs_workspace_bytes(n))


def batch_workspace_bytes(graphs: Sequence[DeviceGraph]) -> int:
    arr = (lexbfs_graph_t * len(graphs))(*[g.desc() for g in graphs])
    return int(_lib.load().lexbfs_batch_workspace_bytes(arr, len(graphs)))


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def lexbfs_order(g: DeviceGraph, stream=None, ws: Optional[torch.Tensor] = None):
    """(order, rank, parent) int32 device tensors."""
    lib = _lib.load()
    n = g.n
    dev = g.device
    order = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    rank = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    parent = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    need = int(lib.lexbfs_workspace_bytes(n))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    d = g.desc()
    rc = lib.lexbfs_order(ctypes.byref(d), _ptr(order), _ptr(rank), _ptr(parent), ws.data_ptr(), ws.numel(),
                          _stream_handle(stream))
    _lib.check(rc, "lexbfs_order")
    _on_stream(stream, ws, order, rank, parent)
    return order[:n], rank[:n], parent[:n]


def lexbfs_plus(g: DeviceGraph, prev_order: torch.Tensor, stream=None, ws: Optional[torch.Tensor] = None):
    """One LexBFS+ sweep after `prev_order` (int32 device tensor of n
    vertices): (order, rank, parent) int32 device tensors. Ties go to the
    vertex that comes last in prev_order."""
    lib = _lib.load()
    n = g.n
    dev = g.device
    order = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    rank = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    parent = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    if n > 0 and (prev_order.dtype != torch.int32 or prev_order.numel() != n or not prev_order.is_contiguous()):
        raise ValueError("prev_order must be a contiguous int32 tensor of n entries")
    need = int(lib.lexbfs_plus_workspace_bytes(n, g.nnz))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    d = g.desc()
    rc = lib.lexbfs_plus_order(ctypes.byref(d), _ptr(prev_order) if n > 0 else None, _ptr(order), _ptr(rank),
                               _ptr(parent), ws.data_ptr(), ws.numel(), _stream_handle(stream))
    _lib.check(rc, "lexbfs_plus_order")
    _on_stream(stream, ws, order, rank, parent)
    return order[:n], rank[:n], parent[:n]


@dataclass
class IntervalResult:
    unit_interval: Optional[bool]
    witness: tuple                       # (a, b, c) or (-1, -1, -1)
    order: Optional[torch.Tensor]        # the third sweep (device)
    res_raw: Optional[torch.Tensor] = None


def unit_interval_test(g: DeviceGraph, stream=None, ws: Optional[torch.Tensor] = None,
                       sync: bool = True) -> IntervalResult:
    """Three-sweep unit interval test (LexBFS, LexBFS+, LexBFS+, then every
    closed neighbourhood consecutive in the third order). With sync=False
    only res_raw and order are filled; read them after the stream."""
    lib = _lib.load()
    n = g.n
    dev = g.device
    res = torch.empty(8, dtype=torch.int32, device=dev)
    order = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    need = int(lib.unit_interval_workspace_bytes(n, g.nnz))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    d = g.desc()
    rc = lib.unit_interval_test(ctypes.byref(d), res.data_ptr(), _ptr(order), ws.data_ptr(), ws.numel(),
                                _stream_handle(stream))
    _lib.check(rc, "unit_interval_test")
    _on_stream(stream, ws, res, order)
    if not sync:
        return IntervalResult(None, (-1, -1, -1), order[:n], res)
    _wait(stream)
    r = res.tolist()
    return IntervalResult(bool(r[0]), (r[1], r[2], r[3]), order[:n], res)


def unit_interval_test_batch(graphs: Sequence[DeviceGraph], stream=None, outputs: bool = False,
                             ws: Optional[torch.Tensor] = None, sync: bool = True) -> List[IntervalResult]:
    """unit_interval_test on every graph, batched (one launch per step for
    the whole batch). With outputs=True each result carries its third
    order; with sync=False only res_raw (a row of the shared verdict tensor)
    and order are filled."""
    lib = _lib.load()
    count = len(graphs)
    if count == 0:
        return []
    dev = graphs[0].device
    descs = (lexbfs_graph_t * count)(*[g.desc() for g in graphs])
    res = torch.empty((count, 8), dtype=torch.int32, device=dev)
    orders = [torch.empty(max(g.n, 1), dtype=torch.int32, device=dev) for g in graphs] if outputs else None
    optr = (ctypes.c_void_p * count)(*[o.data_ptr() for o in orders]) if outputs else None
    need = int(lib.unit_interval_batch_workspace_bytes(descs, count))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    rc = lib.unit_interval_test_batch(descs, count, res.data_ptr(), optr, ws.data_ptr(), ws.numel(),
                                      _stream_handle(stream))
    _lib.check(rc, "unit_interval_test_batch")
    _on_stream(stream, ws, res, *(orders or []))
    out = []
    if sync:
        _wait(stream)
    rows = res.tolist() if sync else None
    for i, g in enumerate(graphs):
        order = orders[i][:g.n] if outputs else None
        if sync:
            r = rows[i]
            out.append(IntervalResult(bool(r[0]), (r[1], r[2], r[3]), order, res[i]))
        else:
            out.append(IntervalResult(None, (-1, -1, -1), order, res[i]))
    return out


def _result_from(row: torch.Tensor) -> tuple:
    r = row.tolist()
    return bool(r[0]), (r[1], r[2], r[3]), r[4], bool(r[5])


def chordal_test(g: DeviceGraph, flags: int = 0, stream=None, outputs: bool = True,
                 ws: Optional[torch.Tensor] = None, sync: bool = True) -> Result:
    """Run the whole test on one graph. With sync=False the returned Result
    holds only device tensors (res_raw) and must be read after the stream."""
    lib = _lib.load()
    n = g.n
    dev = g.device
    res = _zeros_on(8, dev, stream)
    outs = lexbfs_outputs_t()
    tens = {}
    if outputs:
        for k in ("order", "rank", "parent", "cycle"):
            tens[k] = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
            setattr(outs, k, tens[k].data_ptr())
    need = int(lib.lexbfs_workspace_bytes(n))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    d = g.desc()
    rc = lib.chordal_test(ctypes.byref(d), res.data_ptr(), ctypes.byref(outs), ws.data_ptr(), ws.numel(),
                          flags, _stream_handle(stream))
    _lib.check(rc, "chordal_test")
    _on_stream(stream, ws, res, *tens.values())
    if not sync:
        r = Result(False, (-1, -1, -1), 0, False, **{k: v[:n] for k, v in tens.items()})
        r.res_raw = res
        return r
    _wait(stream)
    chordal, wit, clen, fb = _result_from(res.cpu())
    return Result(chordal, wit, clen, fb, **{k: v[:n] for k, v in tens.items()})


def chordal_test_noalloc(g: DeviceGraph, res: torch.Tensor, outputs: Optional[dict] = None, flags: int = 0,
                         stream=None) -> None:
    """chordal_test with the library's fixed per-device scratch array instead
    of a workspace: nothing is allocated on the call's path. The caller
    passes the int32 result record `res` (8 entries, device) and optionally
    int32 [n] device tensors keyed order, rank, parent and cycle; they are
    valid once `stream` has reached the call (Result.from_record reads res).
    Calls that overlap on one device share the array and race."""
    lib = _lib.load()
    outs = lexbfs_outputs_t()
    tens = []
    for k, v in (outputs or {}).items():
        if k not in ("order", "rank", "parent", "cycle"):
            raise ValueError(f"unknown output {k!r}")
        setattr(outs, k, v.data_ptr())
        tens.append(v)
    d = g.desc()
    rc = lib.chordal_test_noalloc(ctypes.byref(d), res.data_ptr(), ctypes.byref(outs), flags,
                                  _stream_handle(stream))
    _lib.check(rc, "chordal_test_noalloc")
    _on_stream(stream, res, *tens)


def chordal_test_noalloc_max_bytes() -> int:
    return int(_lib.load().chordal_test_noalloc_max_bytes())


def chordal_test_batch(graphs: Sequence[DeviceGraph], flags: int = 0, stream=None, outputs: bool = False,
                       tuning: Optional[dict] = None, ws: Optional[torch.Tensor] = None,
                       res: Optional[torch.Tensor] = None, sync: bool = True):
    """Run the test on many graphs in one pass. Returns a list of Result
    (with per-graph order/rank/parent/cycle tensors if outputs=True)."""
    lib = _lib.load()
    count = len(graphs)
    if count == 0:
        return []
    dev = graphs[0].device
    arr = (lexbfs_graph_t * count)(*[g.desc() for g in graphs])
    outs_arr = None
    tens = []
    if outputs:
        outs_arr = (lexbfs_outputs_t * count)()
        for i, g in enumerate(graphs):
            t = {k: torch.empty(max(g.n, 1), dtype=torch.int32, device=dev) for k in ("order", "rank", "parent", "cycle")}
            tens.append(t)
            for k, v in t.items():
                setattr(outs_arr[i], k, v.data_ptr())
    if res is None:
        res = _zeros_on((count, 8), dev, stream)
    need = int(lib.lexbfs_batch_workspace_bytes(arr, count))
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    tun = None
    if tuning:
        tun = lexbfs_tuning_t()
        tun.wave_max_n = int(tuning.get("wave_max_n", 0))
        tun.block_threads = int(tuning.get("block_threads", 0))
        tun.lds_bytes = int(tuning.get("lds_bytes", 0))
        tun = ctypes.byref(tun)
    rc = lib.chordal_test_batch(arr, count, outs_arr, res.data_ptr(), tun, ws.data_ptr(), ws.numel(), flags,
                                _stream_handle(stream))
    _lib.check(rc, "chordal_test_batch")
    _on_stream(stream, ws, res, *(t for d in tens for t in d.values()))
    if not sync:
        return res
    _wait(stream)
    host = res.cpu()
    out = []
    for i, g in enumerate(graphs):
        chordal, wit, clen, fb = _result_from(host[i])
        kw = {k: v[: g.n] for k, v in tens[i].items()} if outputs else {}
        out.append(Result(chordal, wit, clen, fb, **kw))
    return out


def pack_graphs(graphs, device="cuda") -> List[DeviceGraph]:
    """Upload many host graphs with three copies: one pool each for row
    pointers, column indices and bitsets; every DeviceGraph is a view into
    the pools. Bitsets start on 16-byte boundaries."""
    import numpy as np

    rp_off, ci_off, b_off = [0], [0], [0]
    for g in graphs:
        rp_off.append(rp_off[-1] + g.n + 1)
        ci_off.append(ci_off[-1] + max(g.nnz, 0))
        nb = max(g.n * g.W, 1)
        b_off.append(b_off[-1] + nb + (nb & 1))
    rp = np.empty(rp_off[-1], dtype=np.int32)
    ci = np.empty(max(ci_off[-1], 1), dtype=np.int32)
    bits = np.zeros(max(b_off[-1], 1), dtype=np.uint64)
    for i, g in enumerate(graphs):
        rp[rp_off[i]:rp_off[i + 1]] = g.row_ptr
        ci[ci_off[i]:ci_off[i + 1]] = g.col_idx[: g.nnz]
        nb = g.n * g.W
        bits[b_off[i]:b_off[i] + nb] = g.bits[:nb]
    t_rp = torch.from_numpy(rp).to(device)
    t_ci = torch.from_numpy(ci).to(device)
    t_b = torch.from_numpy(bits.view(np.int64)).to(device)
    out = []
    for i, g in enumerate(graphs):
        out.append(DeviceGraph(g.n, g.W, t_rp[rp_off[i]:rp_off[i + 1]], t_ci[ci_off[i]:ci_off[i] + g.nnz],
                               t_b[b_off[i]:b_off[i] + max(g.n * g.W, 1)]))
    return out


class BatchPlan:
    """A prepared batch (lexbfs_batch_plan_*): the schedule and descriptor
    table are built once; launch() only launches the kernels, so it is cheap
    to repeat and may be captured into a HIP graph."""

    def __init__(self, graphs: Sequence[DeviceGraph], outputs: bool = False, tuning: Optional[dict] = None,
                 flags: int = 0, stream=None):
        lib = _lib.load()
        self.graphs = list(graphs)
        count = len(self.graphs)
        dev = self.graphs[0].device if count else torch.device("cuda")
        self.arr = (lexbfs_graph_t * max(count, 1))(*[g.desc() for g in self.graphs])
        self.tens = []
        self.outs_arr = None
        if outputs and count:
            self.outs_arr = (lexbfs_outputs_t * count)()
            for i, g in enumerate(self.graphs):
                t = {k: torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)
                     for k in ("order", "rank", "parent", "cycle")}
                self.tens.append(t)
                for k, v in t.items():
                    setattr(self.outs_arr[i], k, v.data_ptr())
        # every launch writes every record, so no clearing kernel is needed
        self.res = torch.empty((max(count, 1), 8), dtype=torch.int32, device=dev)
        need = int(lib.lexbfs_batch_workspace_bytes(self.arr, count))
        self.ws = _workspace(need, dev)
        tun = None
        if tuning:
            t = lexbfs_tuning_t()
            t.wave_max_n = int(tuning.get("wave_max_n", 0))
            t.block_threads = int(tuning.get("block_threads", 0))
            t.lds_bytes = int(tuning.get("lds_bytes", 0))
            self._tun = t
            tun = ctypes.byref(t)
        self.handle = ctypes.c_void_p()
        self._streams = set()
        rc = lib.lexbfs_batch_plan_create(self.arr, count, self.outs_arr, self.res.data_ptr(), tun,
                                          self.ws.data_ptr(), self.ws.numel(), flags, _stream_handle(stream),
                                          ctypes.byref(self.handle))
        _lib.check(rc, "lexbfs_batch_plan_create")

    def launch(self, stream=None):
        rc = _lib.load().lexbfs_batch_plan_launch(self.handle, _stream_handle(stream))
        _lib.check(rc, "lexbfs_batch_plan_launch")
        if stream is not None and stream not in self._streams:
            # The plan's tensors are freed with the plan; kernels may still
            # run on this stream then.
            self._streams.add(stream)
            _on_stream(stream, self.ws, self.res, *(t for d in self.tens for t in d.values()))

    def capture(self, stream=None) -> "torch.cuda.CUDAGraph":
        """Record one launch of this plan into a HIP graph (kernel nodes only:
        the launch issues no memset or copy). Replaying the graph is the same
        launch; results are read as after launch(). Capturing turns the
        library's kernel timing (KernelTimer) off: its events are host-side
        bookkeeping that a replay would not update."""
        if _lib.load().lexbfs_profile_enable(0) != 0:
            raise LexbfsError(-1, "disabling kernel timing before capture")
        stream = stream or torch.cuda.Stream(device=self.res.device)
        stream.wait_stream(torch.cuda.current_stream(self.res.device))
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            self.launch()
        torch.cuda.current_stream(self.res.device).wait_stream(stream)
        return graph

    def results(self) -> List[Result]:
        host = self.res.cpu()
        out = []
        for i, g in enumerate(self.graphs):
            chordal, wit, clen, fb = _result_from(host[i])
            kw = {k: v[: g.n] for k, v in self.tens[i].items()} if self.tens else {}
            out.append(Result(chordal, wit, clen, fb, **kw))
        return out

    def close(self):
        if self.handle:
            _lib.load().lexbfs_batch_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
