"""CPU oracle for the LexBFS chordality test -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never loads it and
shares no code with it.

The arithmetic lives in ``oracle.c`` (plain sequential C, built with gcc):

* :func:`lexbfs`      -- partition-refinement LexBFS (Section 4.2) with the
  smallest-id tie-break; returns order, rank and the parent p(v).
* :func:`mcs`         -- Maximum Cardinality Search (Section 5.1) with the
  smallest-id tie-break, by a heap of (label, id) entries.
* :func:`peo`         -- the parent-based perfect-elimination test
  (Section 5.2 box), every failing vertex and the canonical witness.
* :func:`certificate` -- the canonical chordless cycle (project rule; its
  parity is pinned by invariants and brute force, not by the paper).
* :func:`bitset_from_csr` -- the packed adjacency bitset from a CSR, by its
  definition (the input format of Section 6.3, checked against the device
  builder).
* :func:`lexbfs_plus`, :func:`unit_interval_test` -- multi-sweep LexBFS
  (ties to the vertex last in the previous order) and the three-sweep test
  for unit interval graphs (a step towards interval recognition, which the
  paper names as future work).
* :func:`chordal_test` -- all three for one graph (``ordering="mcs"``: the
  same test on the MCS order, Theorem 5.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.oracle_lexbfs.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, i32p]
    lib.oracle_peo.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, u8p, i32p]
    lib.oracle_certificate.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, i32p, i32p, i32p]
    lib.oracle_chordal_test.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, i32p, i32p, i32p]
    lib.oracle_mcs.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, i32p]
    lib.oracle_chordal_test_mcs.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p, i32p, i32p, i32p]
    _lib = lib
    return lib


def _p(a: np.ndarray, ct=ctypes.c_int32):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.int32)
    return rp, ci


@dataclass
class OrderResult:
    order: np.ndarray
    rank: np.ndarray
    parent: np.ndarray


@dataclass
class PeoResult:
    is_peo: bool
    p: np.ndarray
    fail: np.ndarray
    witness: tuple  # (v*, x*, z*) or (-1, -1, -1)


@dataclass
class TestResult:
    chordal: bool
    witness: tuple
    cycle: np.ndarray  # empty when chordal
    fallback: bool
    order: np.ndarray
    rank: np.ndarray
    parent: np.ndarray


def lexbfs(g) -> OrderResult:
    n = g.n
    rp, ci = _csr(g)
    order = np.zeros(max(n, 1), dtype=np.int32)
    rank = np.zeros(max(n, 1), dtype=np.int32)
    parent = np.zeros(max(n, 1), dtype=np.int32)
    rc = _load().oracle_lexbfs(n, _p(rp), _p(ci), _p(order), _p(rank), _p(parent))
    if rc != 0:
        raise RuntimeError(f"oracle_lexbfs failed ({rc})")
    return OrderResult(order[:n], rank[:n], parent[:n])


def mcs(g) -> OrderResult:
    n = g.n
    rp, ci = _csr(g)
    order = np.zeros(max(n, 1), dtype=np.int32)
    rank = np.zeros(max(n, 1), dtype=np.int32)
    parent = np.zeros(max(n, 1), dtype=np.int32)
    rc = _load().oracle_mcs(n, _p(rp), _p(ci), _p(order), _p(rank), _p(parent))
    if rc != 0:
        raise RuntimeError(f"oracle_mcs failed ({rc})")
    return OrderResult(order[:n], rank[:n], parent[:n])


def bitset_from_csr(n: int, row_ptr: np.ndarray, col_idx: np.ndarray, words_per_row: int) -> np.ndarray:
    """The packed adjacency bitset by its definition: bit u (word u // 64,
    bit u % 64) of row v is set iff u is in v's CSR row; uint64[n, W].
    A CSR that names a vertex outside 0..n-1, or whose row pointers are not
    a non-decreasing sequence from 0, describes no graph on n vertices
    (Section 3.1): ValueError."""
    if words_per_row < (n + 63) // 64:
        raise ValueError("words_per_row below ceil(n / 64)")
    rp = np.asarray(row_ptr[: n + 1], dtype=np.int64)
    if len(rp) != n + 1 or (n >= 0 and rp[0] != 0) or np.any(np.diff(rp) < 0) or rp[-1] > len(col_idx):
        raise ValueError("row pointers are not a non-decreasing sequence from 0 within col_idx")
    bits = np.zeros((n, words_per_row), dtype=np.uint64)
    rows = np.repeat(np.arange(n), np.diff(rp))
    cols = np.asarray(col_idx[: len(rows)], dtype=np.int64)
    if cols.size and (cols.min() < 0 or cols.max() >= n):
        raise ValueError("a column index names a vertex outside 0..n-1")
    np.bitwise_or.at(bits, (rows, cols // 64), np.left_shift(np.uint64(1), (cols % 64).astype(np.uint64)))
    return bits


def _relabelled_csr(g, new_id: np.ndarray):
    """CSR of g with vertex v renamed new_id[v], rows ascending."""
    n = g.n
    src = np.repeat(np.arange(n), np.diff(np.asarray(g.row_ptr, dtype=np.int64)))
    a = new_id[src]
    b = new_id[np.asarray(g.col_idx[: len(src)], dtype=np.int64)]
    key = np.lexsort((b, a))
    a, b = a[key], b[key]
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, a + 1, 1)
    return np.cumsum(rp).astype(np.int32), b.astype(np.int32)


class _Csr:
    def __init__(self, n, row_ptr, col_idx):
        self.n, self.row_ptr, self.col_idx = n, row_ptr, col_idx


def lexbfs_plus(g, prev_order: np.ndarray) -> OrderResult:
    """LexBFS+ (the '+' rule of multi-sweep LexBFS): among the unnumbered
    vertices of largest label, the one that comes last in prev_order. With
    new_id(v) = n - 1 - position of v in prev_order, that is the smallest
    new id, so this runs :func:`lexbfs` on the renamed graph and maps the
    order back."""
    n = g.n
    pos = np.empty(n, dtype=np.int64)
    pos[np.asarray(prev_order, dtype=np.int64)] = np.arange(n)
    new_id = n - 1 - pos
    old_of = np.empty(n, dtype=np.int64)
    old_of[new_id] = np.arange(n)
    rp, ci = _relabelled_csr(g, new_id)
    r = lexbfs(_Csr(n, rp, ci))
    order = old_of[r.order].astype(np.int32)
    rank = np.empty(n, dtype=np.int32)
    rank[order] = np.arange(n, dtype=np.int32)
    parent = np.where(r.parent[new_id] >= 0, old_of[np.maximum(r.parent[new_id], 0)], -1).astype(np.int32)
    return OrderResult(order, rank, parent)


@dataclass
class UnitIntervalResult:
    unit_interval: bool
    order: np.ndarray   # the third sweep
    witness: tuple      # (a, b, c): a < b < c in the order, ac an edge, ab or bc not; or (-1, -1, -1)


def unit_interval_test(g) -> UnitIntervalResult:
    """Three sweeps -- LexBFS, then LexBFS+ twice -- and the test that every
    closed neighbourhood is consecutive in the third order (a unit interval
    ordering: u < v < w and uw an edge imply uv and vw edges). Witness: the
    earliest vertex v whose closed neighbourhood is not consecutive, b the
    earliest non-neighbour between its first and last closed neighbour, and
    the triple (first, b, v) if b comes before v, else (v, b, last)."""
    n = g.n
    s1 = lexbfs(g).order
    s2 = lexbfs_plus(g, s1).order
    s3 = lexbfs_plus(g, s2).order
    pos = np.empty(n, dtype=np.int64)
    pos[s3] = np.arange(n)
    for i in range(n):
        v = int(s3[i])
        nbrs = g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]
        ps = np.concatenate([pos[nbrs], [i]])
        lo, hi = int(ps.min()), int(ps.max())
        if hi - lo + 1 == len(ps):
            continue
        inside = np.zeros(hi - lo + 1, dtype=bool)
        inside[ps - lo] = True
        b_pos = lo + int(np.argmin(inside))
        b = int(s3[b_pos])
        if b_pos < i:
            return UnitIntervalResult(False, s3, (int(s3[lo]), b, v))
        return UnitIntervalResult(False, s3, (v, b, int(s3[hi])))
    return UnitIntervalResult(True, s3, (-1, -1, -1))


def peo(g, rank: np.ndarray) -> PeoResult:
    n = g.n
    rp, ci = _csr(g)
    rk = np.ascontiguousarray(rank, dtype=np.int32)
    if rk.size == 0:
        rk = np.zeros(1, dtype=np.int32)
    p = np.zeros(max(n, 1), dtype=np.int32)
    fail = np.zeros(max(n, 1), dtype=np.uint8)
    w = np.full(3, -1, dtype=np.int32)
    rc = _load().oracle_peo(n, _p(rp), _p(ci), _p(rk), _p(p), _p(fail, ctypes.c_uint8), _p(w))
    if rc < 0:
        raise RuntimeError(f"oracle_peo failed ({rc})")
    return PeoResult(rc == 1, p[:n], fail[:n].astype(bool), tuple(int(x) for x in w))


def certificate(g, order, rank, witness, force_fallback: bool = False):
    """Returns (cycle array, used_fallback)."""
    n = g.n
    rp, ci = _csr(g)
    cyc = np.zeros(max(n, 1), dtype=np.int32)
    ln = np.zeros(1, dtype=np.int32)
    fb = np.zeros(1, dtype=np.int32)
    o = np.ascontiguousarray(order, dtype=np.int32)
    r = np.ascontiguousarray(rank, dtype=np.int32)
    v, x, z = witness
    rc = _load().oracle_certificate(n, _p(rp), _p(ci), _p(o), _p(r), v, x, z, int(force_fallback), _p(cyc), _p(ln), _p(fb))
    if rc != 0:
        raise RuntimeError(f"oracle_certificate failed ({rc}): no chordless cycle found")
    return cyc[: int(ln[0])].copy(), bool(fb[0])


def chordal_test(g, ordering: str = "lexbfs") -> TestResult:
    if ordering not in ("lexbfs", "mcs"):
        raise ValueError(f"unknown ordering {ordering!r}")
    n = g.n
    rp, ci = _csr(g)
    m = max(n, 1)
    order = np.zeros(m, dtype=np.int32)
    rank = np.zeros(m, dtype=np.int32)
    parent = np.zeros(m, dtype=np.int32)
    cyc = np.zeros(m, dtype=np.int32)
    res = np.zeros(6, dtype=np.int32)
    fn = _load().oracle_chordal_test if ordering == "lexbfs" else _load().oracle_chordal_test_mcs
    rc = fn(n, _p(rp), _p(ci), _p(order), _p(rank), _p(parent), _p(cyc), _p(res))
    if rc != 0:
        raise RuntimeError(f"oracle_chordal_test failed ({rc})")
    return TestResult(bool(res[0]), (int(res[1]), int(res[2]), int(res[3])), cyc[: int(res[4])].copy(),
                      bool(res[5]), order[:n], rank[:n], parent[:n])


class use_library:
    """Context manager: route this module's calls to another build of
    oracle.c (tests use it to check that planted mistakes are caught)."""

    def __init__(self, path: str):
        self.path = path
        self.saved = None

    def __enter__(self):
        global _lib, _LIB_PATH
        self.saved = (_lib, _LIB_PATH)
        _lib, _LIB_PATH = None, self.path
        _load()
        return self

    def __exit__(self, *exc):
        global _lib, _LIB_PATH
        _lib, _LIB_PATH = self.saved
        return False
