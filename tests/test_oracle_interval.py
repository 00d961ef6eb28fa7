"""Pins of the oracle's multi-sweep LexBFS+ and of the three-sweep unit
interval test (CPU only): the literal label definition with the '+' rule,
brute force over all vertex orders, and claws in generated interval graphs."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from brute import (all_graphs, closed_nbhds_consecutive, has_induced_claw, lexbfs_plus_by_labels,
                   unit_interval_by_orderings)


def graph(n, adj):
    return gg.from_edges(n, [(a, b) for a in range(n) for b in adj[a] if a < b])


def check_witness(g, r):
    adj = [set(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(g.n)]
    if r.unit_interval:
        assert closed_nbhds_consecutive(r.order.tolist(), adj)
        return
    a, b, c = r.witness
    pos = {v: i for i, v in enumerate(r.order.tolist())}
    assert pos[a] < pos[b] < pos[c] and c in adj[a] and (b not in adj[a] or c not in adj[b])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_every_small_graph(n):
    rng = np.random.default_rng(n)
    for mask, pairs, adj in all_graphs(n):
        g = graph(n, adj)
        prev = rng.permutation(n)
        assert oracle.lexbfs_plus(g, prev).order.tolist() == lexbfs_plus_by_labels(n, adj, prev.tolist()), mask
        r = oracle.unit_interval_test(g)
        assert r.unit_interval == unit_interval_by_orderings(n, adj), (n, mask)
        check_witness(g, r)


@pytest.mark.parametrize("n", [6, 7])
def test_random_small_graphs(n):
    rng = np.random.default_rng(10 + n)
    for trial in range(150):
        p = rng.uniform(0.2, 0.8)
        M = np.triu(rng.random((n, n)) < p, 1)
        adj = [set() for _ in range(n)]
        for a, b in zip(*np.nonzero(M)):
            adj[int(a)].add(int(b))
            adj[int(b)].add(int(a))
        g = graph(n, adj)
        prev = rng.permutation(n)
        assert oracle.lexbfs_plus(g, prev).order.tolist() == lexbfs_plus_by_labels(n, adj, prev.tolist())
        r = oracle.unit_interval_test(g)
        assert r.unit_interval == unit_interval_by_orderings(n, adj), trial
        check_witness(g, r)


@pytest.mark.parametrize("seed", range(4))
def test_generated_interval_graphs(seed):
    """Unit interval graphs are recognised (with a consecutive-neighbourhood
    order as proof); interval graphs from mixed lengths are rejected exactly
    when they contain an induced claw (Roberts: unit interval = interval and
    claw-free)."""
    for n, deg in ((60, 4), (300, 6), (1000, 8)):
        g = gg.intervals(n, deg, 100 * seed + n)
        r = oracle.unit_interval_test(g)
        assert r.unit_interval
        check_witness(g, r)
        h = gg.intervals(n, deg, 100 * seed + n + 1, unit=False)
        adj = [set(h.col_idx[h.row_ptr[v]:h.row_ptr[v + 1]].tolist()) for v in range(n)]
        r = oracle.unit_interval_test(h)
        assert r.unit_interval == (not has_induced_claw(n, adj))
        check_witness(h, r)


def test_families():
    assert oracle.unit_interval_test(gg.from_edges(7, [(i, i + 1) for i in range(6)])).unit_interval
    assert oracle.unit_interval_test(gg.from_edges(6, [(a, b) for a in range(6) for b in range(a + 1, 6)])).unit_interval
    assert not oracle.unit_interval_test(gg.from_edges(4, [(0, 1), (0, 2), (0, 3)])).unit_interval  # claw
    assert not oracle.unit_interval_test(gg.from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)])).unit_interval  # C4
    # disjoint union of a path and a triangle, ids interleaved
    g = gg.from_edges(7, [(0, 2), (2, 4), (4, 6), (1, 3), (3, 5), (5, 1)])
    assert oracle.unit_interval_test(g).unit_interval
