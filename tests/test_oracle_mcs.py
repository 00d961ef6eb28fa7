"""Pins of the oracle's Maximum Cardinality Search (Section 5.1) and of the
chordality test on its order (Theorem 5.2), against what the definitions
and the theorem fix (CPU only)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from brute import (all_graphs, chordal_by_holes, is_chordless_cycle, is_peo_full, mcs_by_counts, random_adj,
                   witness_by_definition, certificate_by_enumeration)


def graph(n, adj):
    return gg.from_edges(n, [(a, b) for a in range(n) for b in adj[a] if a < b])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_every_small_graph(n):
    """Order = the counting definition; verdict = hole enumeration
    (Theorem 5.2); certificate = a chordless cycle, the enumerated one."""
    for mask, pairs, adj in all_graphs(n):
        g = graph(n, adj)
        r = oracle.chordal_test(g, "mcs")
        assert r.order.tolist() == mcs_by_counts(n, adj), (n, mask)
        assert r.chordal == chordal_by_holes(n, adj), (n, mask)
        assert r.chordal == is_peo_full(r.order.tolist(), adj), (n, mask)
        if not r.chordal:
            assert tuple(r.witness) == witness_by_definition(r.order.tolist(), adj), (n, mask)
            assert is_chordless_cycle(r.cycle.tolist(), adj), (n, mask)
            if not r.fallback:
                assert r.cycle.tolist() == certificate_by_enumeration(n, adj, *r.witness), (n, mask)


@pytest.mark.parametrize("n", [4, 5, 8, 33, 100])
def test_closed_forms(n):
    cyc = gg.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    # every count ties at 1 until the last vertex: the smallest id wins each time
    assert oracle.mcs(cyc).order.tolist() == list(range(n))
    assert oracle.lexbfs(cyc).order.tolist() != list(range(n))  # LexBFS distinguishes the two ends
    k = gg.from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
    assert oracle.mcs(k).order.tolist() == list(range(n))
    c = n // 2
    star = gg.from_edges(n, [(c, v) for v in range(n) if v != c])
    assert oracle.mcs(star).order.tolist() == [0, c] + [v for v in range(1, n) if v != c]
    path = gg.from_edges(n, [(i, i + 1) for i in range(n - 1)])
    assert oracle.mcs(path).order.tolist() == list(range(n))
    assert not oracle.chordal_test(cyc, "mcs").chordal and oracle.chordal_test(k, "mcs").chordal


@pytest.mark.parametrize("seed", range(6))
def test_maximum_cardinality_property_and_parents(seed):
    """Each pivot has the most numbered neighbours among the unnumbered
    vertices (smallest id on ties), and p(v) is v's latest earlier
    neighbour -- checked step by step on larger random graphs."""
    rng = np.random.default_rng(seed)
    n = 150
    adj = random_adj(n, 0.05 + 0.02 * seed, rng)
    r = oracle.mcs(graph(n, adj))
    cnt = np.zeros(n, dtype=int)
    numbered = np.zeros(n, dtype=bool)
    for i, x in enumerate(r.order.tolist()):
        cand = [(-cnt[v], v) for v in range(n) if not numbered[v]]
        assert min(cand) == (-cnt[x], x), (seed, i)
        numbered[x] = True
        for y in adj[x]:
            if not numbered[y]:
                cnt[y] += 1
        earlier = [u for u in adj[x] if r.rank[u] < i]
        assert r.parent[x] == (max(earlier, key=lambda u: r.rank[u]) if earlier else -1)


@pytest.mark.parametrize("seed", range(4))
def test_verdicts_match_lexbfs_and_certificates_are_chordless(seed):
    for g in (gg.subtree(400, 100, 6, seed), gg.plant(gg.subtree(300, 80, 6, seed), 5 + seed, seed),
              gg.gnp(200, 0.03, seed), gg.split_pair(30, 200, 5, seed)[1]):
        a, b = oracle.chordal_test(g, "mcs"), oracle.chordal_test(g)
        assert a.chordal == b.chordal, g.name
        if not a.chordal:
            adj = [set(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(g.n)]
            assert is_chordless_cycle(a.cycle.tolist(), adj) and len(a.cycle) >= 4
            assert a.cycle[0] == a.witness[0] and a.cycle[1] == a.witness[1] and a.cycle[-1] == a.witness[2]
