"""Seeded synthetic graph inputs (host side).

Inputs only: this package holds none of the chordality method's arithmetic.
Every generator returns a :class:`Graph` holding both layouts the library
consumes -- an N x N LSB-first uint64 adjacency bitset with row stride ``W``
words, and a sorted symmetric int32 CSR derived from it.

The generators follow the workload shapes of the paper's test classes
(cliques, trees, sparse and dense random graphs, chordal random graphs;
Section 7) and the batch/serving mixes built on them:

* ``subtree(n, T, smax)``  -- intersection graph of random subtrees of a
  uniform random labelled tree (chordal by construction);
* ``gnp(n, p)``            -- Erdos-Renyi G(n, p);
* ``split(K, I, a)``       -- a K-clique plus I independent vertices, each
  joined to a uniform a-subset of the clique (chordal);
* ``plant(g, L)``          -- append a chordless L-cycle bridged to one
  existing vertex (non-chordal for L >= 4).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with gcc (host code only)."""
    import subprocess

    src = os.path.join(_HERE, "graphgen.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.gg_graph_seed.restype = ctypes.c_uint64
    lib.gg_graph_seed.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_rng_stream.argtypes = [ctypes.c_uint64, ctypes.c_int64, u64p]
    lib.gg_splitmix_stream.argtypes = [ctypes.c_uint64, ctypes.c_int64, u64p]
    for name in ("gg_subtree",):
        getattr(lib, name).argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, u64p, ctypes.c_int64]
    lib.gg_gnp.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_uint64, u64p, ctypes.c_int64]
    lib.gg_split.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, u64p, ctypes.c_int64]
    lib.gg_plant.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, u64p, ctypes.c_int64]
    lib.gg_bits_nnz.restype = ctypes.c_int64
    lib.gg_bits_nnz.argtypes = [ctypes.c_int, u64p, ctypes.c_int64]
    lib.gg_bits_to_csr.argtypes = [ctypes.c_int, u64p, ctypes.c_int64, i32p, i32p]
    lib.gg_edges_to_bits.argtypes = [ctypes.c_int, ctypes.c_int64, i32p, i32p, u64p, ctypes.c_int64]
    lib.gg_permutation.argtypes = [ctypes.c_int, ctypes.c_uint64, i32p]
    lib.gg_mix_draws.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_double, i32p, i32p, f64p]
    lib.gg_mix_types.argtypes = [ctypes.c_uint64, ctypes.c_int64, i32p]
    _lib = lib
    return lib


def _p(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


@dataclass
class Graph:
    """A simple undirected graph in both layouts.

    ``bits``: uint64[n * W], row v = bits[v*W:(v+1)*W], LSB-first.
    ``row_ptr``: int32[n+1]; ``col_idx``: int32[nnz], ascending per row.
    """

    n: int
    W: int
    bits: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def neighbors(self, v: int) -> np.ndarray:
        return self.col_idx[self.row_ptr[v]:self.row_ptr[v + 1]]

    def has_edge(self, u: int, v: int) -> bool:
        return bool((int(self.bits[u * self.W + (v >> 6)]) >> (v & 63)) & 1)

    def adj_sets(self) -> List[set]:
        return [set(int(x) for x in self.neighbors(v)) for v in range(self.n)]


def words_for(n: int) -> int:
    return max(1, (n + 63) // 64)


def empty_bits(n: int, W: Optional[int] = None) -> Tuple[np.ndarray, int]:
    W = words_for(n) if W is None else W
    return np.zeros(max(1, n * W), dtype=np.uint64), W


def finish(n: int, bits: np.ndarray, W: int, name: str = "", **meta) -> Graph:
    """Derive the CSR from a filled bitset."""
    lib = _load()
    nnz = int(lib.gg_bits_nnz(n, _p(bits, ctypes.c_uint64), W))
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    col_idx = np.zeros(max(nnz, 1), dtype=np.int32)
    rc = lib.gg_bits_to_csr(n, _p(bits, ctypes.c_uint64), W, _p(row_ptr, ctypes.c_int32), _p(col_idx, ctypes.c_int32))
    if rc != 0:
        raise ValueError("graph too large for int32 CSR")
    return Graph(n, W, bits, row_ptr, col_idx[:nnz], name, dict(meta))


def graph_seed(config_seed: int, index: int) -> int:
    return int(_load().gg_graph_seed(config_seed, index))


def rng_stream(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    _load().gg_rng_stream(seed, count, _p(out, ctypes.c_uint64))
    return out


def splitmix_stream(state: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    _load().gg_splitmix_stream(state, count, _p(out, ctypes.c_uint64))
    return out


def from_edges(n: int, edges: Sequence[Tuple[int, int]], name: str = "") -> Graph:
    bits, W = empty_bits(n)
    if len(edges):
        e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
        eu = np.ascontiguousarray(e[:, 0])
        ev = np.ascontiguousarray(e[:, 1])
        rc = _load().gg_edges_to_bits(n, len(eu), _p(eu, ctypes.c_int32), _p(ev, ctypes.c_int32), _p(bits, ctypes.c_uint64), W)
        if rc != 0:
            raise ValueError("bad edge list (out of range or self-loop)")
    return finish(n, bits, W, name)


def from_adjacency(adj: np.ndarray, name: str = "") -> Graph:
    """From a dense symmetric 0/1 matrix (test helper)."""
    n = adj.shape[0]
    iu, ju = np.nonzero(np.triu(adj, 1))
    return from_edges(n, list(zip(iu.tolist(), ju.tolist())), name)


def subtree(n: int, T: int, smax: int, seed: int, n_total: Optional[int] = None) -> Graph:
    n_total = n if n_total is None else n_total
    bits, W = empty_bits(n_total)
    if _load().gg_subtree(n, T, smax, seed, _p(bits, ctypes.c_uint64), W) != 0:
        raise ValueError("gg_subtree failed")
    return finish(n_total, bits, W, f"subtree({n},{T},{smax})", seed=seed)


def gnp(n: int, p: float, seed: int) -> Graph:
    bits, W = empty_bits(n)
    if _load().gg_gnp(n, p, seed, _p(bits, ctypes.c_uint64), W) != 0:
        raise ValueError("gg_gnp failed")
    return finish(n, bits, W, f"gnp({n},{p:g})", seed=seed)


def split(K: int, I: int, a: int, seed: int) -> Graph:
    n = K + I
    bits, W = empty_bits(n)
    if _load().gg_split(K, I, a, seed, _p(bits, ctypes.c_uint64), W) != 0:
        raise ValueError("gg_split failed")
    return finish(n, bits, W, f"split({K},{I},{a})", seed=seed)


def plant_subtree(n: int, L: int, T: int, smax: int, seed_tree: int, seed_plant: int) -> Graph:
    """SUBTREE on the first n-L ids, then PLANT(L) on ids [n-L, n)."""
    n0 = n - L
    bits, W = empty_bits(n)
    lib = _load()
    if lib.gg_subtree(n0, T, smax, seed_tree, _p(bits, ctypes.c_uint64), W) != 0:
        raise ValueError("gg_subtree failed")
    if lib.gg_plant(n0, L, seed_plant, _p(bits, ctypes.c_uint64), W) != 0:
        raise ValueError("gg_plant failed")
    return finish(n, bits, W, f"plant(subtree({n0},{T},{smax}),{L})", seed=seed_tree)


def plant(g: Graph, L: int, seed: int) -> Graph:
    """Copy of g with a chordless L-cycle on L new ids bridged to one old vertex."""
    n = g.n + L
    bits, W = empty_bits(n)
    b2 = bits.reshape(n, W)
    b2[: g.n, : g.W] = g.bits.reshape(g.n, g.W)[:, : min(g.W, W)]
    if _load().gg_plant(g.n, L, seed, _p(bits, ctypes.c_uint64), W) != 0:
        raise ValueError("gg_plant failed")
    return finish(n, bits, W, f"plant({g.name},{L})", seed=seed)


def remove_edge(g: Graph, u: int, v: int) -> Graph:
    bits = g.bits.copy()
    for a, b in ((u, v), (v, u)):
        bits[a * g.W + (b >> 6)] &= np.uint64(~(1 << (b & 63)) & 0xFFFFFFFFFFFFFFFF)
    return finish(g.n, bits, g.W, f"{g.name}-({u},{v})")


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Graph with vertex v renamed perm[v]."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    dst = g.col_idx.astype(np.int64)
    keep = src < dst
    e = np.stack([perm[src[keep]], perm[dst[keep]]], axis=1)
    return from_edges(g.n, e, f"relabel({g.name})")


def permutation(n: int, seed: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.int32)
    _load().gg_permutation(n, seed, _p(out, ctypes.c_int32))
    return out


# ---------------------------------------------------------------------------
# Workload configurations (seed 0 unless stated).
# ---------------------------------------------------------------------------

def intervals(n: int, avg_deg: float, seed: int, unit: bool = True) -> Graph:
    """Intersection graph of n random closed intervals on a line: left ends
    uniform on [0, 2n / avg_deg), length 1 (unit) or uniform on [0, 2), ids
    shuffled by a random permutation (so they do not follow the line)."""
    u = rng_stream(seed, 2 * n).astype(np.float64) / 2.0 ** 64
    span = 2.0 * n / max(avg_deg, 1e-9)
    left = u[:n] * span
    right = left + (1.0 if unit else 2.0 * u[n:])
    idx = np.argsort(left, kind="stable")
    # In left-end order, interval a meets the later intervals b with
    # left[b] <= right[a]: positions a+1 .. hi[a]-1.
    hi = np.searchsorted(left[idx], right[idx], side="right")
    cnt = np.maximum(hi - np.arange(n) - 1, 0)
    src = np.repeat(np.arange(n), cnt)
    first = np.repeat(np.cumsum(cnt) - cnt, cnt)
    dst = src + 1 + (np.arange(int(cnt.sum())) - first)
    edges = np.stack([idx[src], idx[dst]], axis=1).astype(np.int32)
    g = from_edges(n, edges, f"{'unit_' if unit else ''}intervals({n},{avg_deg})")
    return relabel(g, permutation(n, seed + 1))


def config_single_small(seed: int = 0) -> List[Graph]:
    """N = 1,024 subtree graph (host tree 256 nodes, subtree size in [1, 8]),
    and the same graph with a planted chordless 5-cycle (N = 1,029)."""
    g = subtree(1024, 256, 8, graph_seed(seed, 0))
    h = plant(g, 5, graph_seed(seed, 1))
    return [g, h]


def config_single_large(seed: int = 0) -> List[Graph]:
    """N = 16,384 subtree graph (host tree 4,096 nodes, subtree size in
    [1, 16]) and G(16384, 0.003)."""
    return [subtree(16384, 4096, 16, graph_seed(seed, 2)), gnp(16384, 0.003, graph_seed(seed, 3))]


def split_pair(K: int, I: int, a: int, seed: int) -> List[Graph]:
    """SPLIT(K, I, a) and the copy without clique edge (a0, b0), the two
    smallest clique ids adjacent to vertex K. Any clique vertex c outside
    N(K) then closes the hole a0-c-b0-K, so the copy is not chordal."""
    g = split(K, I, a, seed)
    nb = [int(x) for x in g.neighbors(K) if x < K]
    a0, b0 = nb[0], nb[1]
    h = remove_edge(g, a0, b0)
    h.meta["removed"] = (a0, b0)
    return [g, h]


def config_worst_steps(seed: int = 0) -> List[Graph]:
    """N = 65,536 split graph: clique of 4,096 plus 61,440 independent
    vertices with 64 clique neighbours each; and the copy minus one edge."""
    return split_pair(4096, 61440, 64, graph_seed(seed, 4))


def mix_graph(n: int, kind: int, L: int, seed: int) -> Graph:
    """One graph of the batch/serving mix: kind 0 = SUBTREE(n, ceil(n/4), 8);
    1 = GNP(n, 8/(n-1)); 2 = PLANT(SUBTREE(n-L, ceil((n-L)/4), 8), L)."""
    if kind == 0:
        return subtree(n, max(1, math.ceil(n / 4)), 8, seed)
    if kind == 1:
        return gnp(n, min(1.0, 8.0 / max(1, n - 1)), seed)
    n0 = n - L
    return plant_subtree(n, L, max(1, math.ceil(n0 / 4)), 8, seed, seed ^ 0x5DEECE66D)


def mix_specs(count: int, lo: int, hi: int, seed: int):
    """(n, kind, L, gap) per graph for a log-uniform N mix on [lo, hi]."""
    lib = _load()
    ns = np.zeros(count, dtype=np.int32)
    Ls = np.zeros(count, dtype=np.int32)
    gaps = np.zeros(count, dtype=np.float64)
    lib.gg_mix_draws(graph_seed(seed, 100), count, float(lo), float(hi + 1), _p(ns, ctypes.c_int32), _p(Ls, ctypes.c_int32), _p(gaps, ctypes.c_double))
    kinds = np.zeros(count, dtype=np.int32)
    lib.gg_mix_types(graph_seed(seed, 101), count, _p(kinds, ctypes.c_int32))
    return ns, kinds, Ls, gaps


def config_batch(count: int = 4096, lo: int = 32, hi: int = 4096, seed: int = 0) -> List[Graph]:
    """Batch mix: N log-uniform on [lo, hi]; 50% SUBTREE, 25% GNP with average
    degree 8, 25% SUBTREE with a planted chordless cycle of length in [4, 12]."""
    ns, kinds, Ls, _ = mix_specs(count, lo, hi, seed)
    from concurrent.futures import ThreadPoolExecutor

    def one(i):
        return mix_graph(int(ns[i]), int(kinds[i]), int(Ls[i]), graph_seed(seed, 1000 + i))

    # the C generators release the GIL; results are independent of the pool
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, range(count)))


def interval_mix_graph(n: int, kind: int, seed: int) -> Graph:
    """One graph of the interval batch mix, average degree 8: kind 0 = unit
    intervals, 1 = GNP(n, 8/(n-1)), 2 = intervals of mixed lengths."""
    if kind == 1:
        return gnp(n, min(1.0, 8.0 / max(1, n - 1)), seed)
    return intervals(n, 8.0, seed, unit=kind == 0)


def config_interval_batch(count: int = 4096, lo: int = 32, hi: int = 4096, seed: int = 0) -> List[Graph]:
    """Interval batch: the sizes and kind draws of the batch mix (N
    log-uniform on [lo, hi]); 50% unit interval graphs, 25% GNP with average
    degree 8, 25% interval graphs of mixed lengths."""
    ns, kinds, _, _ = mix_specs(count, lo, hi, seed)
    from concurrent.futures import ThreadPoolExecutor

    def one(i):
        return interval_mix_graph(int(ns[i]), int(kinds[i]), graph_seed(seed, 2000 + i))

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, range(count)))
