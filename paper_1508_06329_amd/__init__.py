"""LexBFS chordality test on MI355X (gfx950).

Python binding of ``liblexbfs.so`` (C ABI in ``include/lexbfs.h``). PyTorch
supplies device memory and streams; every step of the path runs in the HIP
kernels: the LexBFS order (Section 6.1 of Lupinska, "A Parallel Algorithm to
Test Chordality of Graphs"), the perfect-elimination test (Section 6.2), and
a chordless-cycle certificate for non-chordal graphs.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import (LEXBFS_FLAG_FORCE_FALLBACK, LEXBFS_MAX_N, LexbfsError, lexbfs_graph_t, lexbfs_outputs_t,
                   lexbfs_result_t, lexbfs_tuning_t)

__all__ = ["DeviceGraph", "Result", "lexbfs_order", "chordal_test", "chordal_test_batch", "workspace_bytes",
           "batch_workspace_bytes", "LexbfsError", "LEXBFS_MAX_N", "LEXBFS_FLAG_FORCE_FALLBACK"]


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> Optional[int]:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


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
    return order[:n], rank[:n], parent[:n]


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
    res = torch.zeros(8, dtype=torch.int32, device=dev)
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
    if not sync:
        r = Result(False, (-1, -1, -1), 0, False, **{k: v[:n] for k, v in tens.items()})
        r.res_raw = res
        return r
    if stream is not None:
        stream.synchronize()
    else:
        torch.cuda.current_stream().synchronize()
    chordal, wit, clen, fb = _result_from(res.cpu())
    return Result(chordal, wit, clen, fb, **{k: v[:n] for k, v in tens.items()})


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
        res = torch.zeros((count, 8), dtype=torch.int32, device=dev)
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
    if not sync:
        return res
    (stream or torch.cuda.current_stream()).synchronize()
    host = res.cpu()
    out = []
    for i, g in enumerate(graphs):
        chordal, wit, clen, fb = _result_from(host[i])
        kw = {k: v[: g.n] for k, v in tens[i].items()} if outputs else {}
        out.append(Result(chordal, wit, clen, fb, **kw))
    return out
