"""Pins of the oracle's multi-sweep LexBFS+ and of the three-sweep unit
interval test (CPU only): the literal label definition with the '+' rule,
brute force over all vertex orders, and claws in generated interval graphs."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from brute import (all_graphs, closed_nbhds_consecutive, has_induced_claw, lexbfs_by_labels, lexbfs_plus_by_labels,
                   parents_by_definition, random_adj, three_sweeps_by_labels, unit_interval_by_orderings,
                   unit_interval_witness_by_definition)


def graph(n, adj):
    return gg.from_edges(n, [(a, b) for a in range(n) for b in adj[a] if a < b])


def adjacency(g):
    return [set(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(g.n)]


def check_witness(g, r):
    """Validity of the verdict and witness, and exact agreement of the third
    order and the witness with the label-string sweeps and the witness rule
    written out from its definition."""
    adj = adjacency(g)
    assert r.order.tolist() == three_sweeps_by_labels(g.n, adj)
    expect = unit_interval_witness_by_definition(r.order.tolist(), adj)
    if r.unit_interval:
        assert expect is None
        assert closed_nbhds_consecutive(r.order.tolist(), adj)
        assert r.witness == (-1, -1, -1)
        return
    assert r.witness == expect
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
    for n, deg in ((60, 4), (300, 6), (600, 8)):
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


def test_witness_rule_by_hand():
    """A claw 0-{1,2,3} with 3-4 attached: worked by hand from the sweeps.
    sigma1 = 0,1,2,3,4 (smallest ids); sigma2 (ties to the latest of sigma1):
    4, 3, 0, 2, 1; sigma3 (ties to the latest of sigma2): 1, 0, 2, 3, 4.
    N[0] = {0,1,2,3} sits on positions 0..3, consecutive; N[1] = {0,1} too;
    N[2] = {0,2} sits on positions 1..2; N[3] = {0,3,4} sits on positions
    1, 3, 4: the first failure, span 1..4, b = the vertex at position 2,
    i.e. 2, which comes before 3: triple (sigma3[1], 2, 3) = (0, 2, 3)."""
    g = gg.from_edges(5, [(0, 1), (0, 2), (0, 3), (3, 4)])
    r = oracle.unit_interval_test(g)
    assert not r.unit_interval
    assert r.order.tolist() == [1, 0, 2, 3, 4]
    assert r.witness == (0, 2, 3)


@pytest.mark.parametrize("n", [100, 160, 200])
def test_lexbfs_plus_against_labels_mid_size(n):
    """LexBFS+ against the literal label definition with the '+' tie rule
    at a hundred or more vertices, after random previous orders and after
    LexBFS orders (the chain the unit interval test uses), on sparse and
    dense random graphs, subtree graphs and interval graphs; the parents
    against the latest-earlier-neighbour definition."""
    rng = np.random.default_rng(n)
    cases = []
    for p in (0.02, 0.08, 0.3):
        cases.append(random_adj(n, p, rng))
    for g in (gg.subtree(n, n // 4, 6, n), gg.intervals(n, 6, n + 1), gg.intervals(n, 6, n + 2, unit=False)):
        cases.append(adjacency(g))
    for adj in cases:
        g = graph(n, adj)
        for prev in (rng.permutation(n).tolist(), lexbfs_by_labels(n, adj)):
            r = oracle.lexbfs_plus(g, np.array(prev, dtype=np.int32))
            assert r.order.tolist() == lexbfs_plus_by_labels(n, adj, prev)
            assert r.parent.tolist() == parents_by_definition(r.order.tolist(), adj)
            assert np.array_equal(r.rank[r.order], np.arange(n))
