"""Pins for the CPU oracle: things the paper and the mathematics fix.

Each pin is independent of the oracle's own code: worked examples derived by
hand (tests/golden), closed forms derived from the Section 4.1 label
definition, brute force by definition on every graph with n <= 6, the
Lemma 4.2 characterisation (Property LB), Theorem 5.1 (verdict equals "no
hole"), and the Section 5.3 claim that the parent-only test equals the full
perfect-elimination test.
"""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle
from brute import (adj_matrix, all_graphs, certificate_by_enumeration, chordal_by_elimination, chordal_by_holes,
                   first_non_simplicial, is_chordless_cycle, witness_by_definition, is_peo_full, lexbfs_by_labels, random_adj,
                   satisfies_b, satisfies_lb, satisfies_lb_fast)
from conftest import load_golden


def graph_of(n, adj):
    edges = [(a, b) for a in range(n) for b in adj[a] if a < b]
    return gg.from_edges(n, edges)


# ---------------------------------------------------------------------------
# Worked examples (tests/golden)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["c4.txt", "c5.txt", "two_triangles.txt"])
def test_golden_examples(name):
    ex = load_golden(name)
    g = gg.from_edges(ex["n"], ex["edges"])
    r = oracle.chordal_test(g)
    assert r.order.tolist() == ex["order"]
    assert r.parent.tolist() == ex["parent"]
    assert r.chordal == ex["chordal"]
    assert list(r.witness) == ex["witness"]
    assert r.cycle.tolist() == ex["cycle"]
    assert not r.fallback


# ---------------------------------------------------------------------------
# Closed forms from the Section 4.1 label definition with smallest-id ties
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 65, 200])
def test_clique_edgeless_path_identity(n):
    K = gg.from_edges(n, list(itertools.combinations(range(n), 2)))
    E = gg.from_edges(n, [])
    P = gg.from_edges(n, [(i, i + 1) for i in range(n - 1)])
    for g in (K, E, P):
        r = oracle.chordal_test(g)
        assert r.order.tolist() == list(range(n))
        assert r.chordal
    # clique: parent of v is v-1; edgeless: none; path: v-1
    assert oracle.lexbfs(K).parent.tolist() == [-1] + list(range(n - 1))
    assert oracle.lexbfs(E).parent.tolist() == [-1] * n
    assert oracle.lexbfs(P).parent.tolist() == [-1] + list(range(n - 1))


@pytest.mark.parametrize("n,c", [(5, 3), (9, 1), (9, 8), (40, 17)])
def test_star_closed_form(n, c):
    # star with centre c > 0: 0 first (a leaf), then c, then the other leaves ascending
    g = gg.from_edges(n, [(c, v) for v in range(n) if v != c])
    r = oracle.lexbfs(g)
    assert r.order.tolist() == [0, c] + [v for v in range(1, n) if v != c]


@pytest.mark.parametrize("n", [4, 5, 6, 7, 10, 33])
def test_cycle_closed_form(n):
    # C_n labelled cyclically: 0, 1, n-1, 2, n-2, 3, ...
    g = gg.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    r = oracle.chordal_test(g)
    expect = [0]
    lo, hi = 1, n - 1
    while lo <= hi:
        expect.append(lo)
        if hi != lo:
            expect.append(hi)
        lo += 1
        hi -= 1
    assert r.order.tolist() == expect
    assert not r.chordal
    assert sorted(r.cycle.tolist()) == list(range(n))  # the only hole is the whole cycle
    assert is_chordless_cycle(r.cycle.tolist(), g.adj_sets())


# ---------------------------------------------------------------------------
# Exhaustive brute force over every labelled graph with n <= 6
# ---------------------------------------------------------------------------

CHORDAL_COUNTS_BY_HAND = {1: 1, 2: 2, 3: 8, 4: 61}   # n=4: 64 graphs minus the 3 labelled C4


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_small(n):
    count = 0
    for mask, pairs, adj in all_graphs(n):
        g = graph_of(n, adj)
        r = oracle.chordal_test(g)
        assert r.order.tolist() == lexbfs_by_labels(n, adj), (n, mask)
        assert satisfies_lb(r.order.tolist(), adj)
        holes = chordal_by_holes(n, adj)
        assert holes == chordal_by_elimination(n, adj)
        assert r.chordal == holes, (n, mask)
        count += holes
        # the parent from LexBFS is the latest earlier neighbour
        pos = {v: i for i, v in enumerate(r.order.tolist())}
        for v in range(n):
            earlier = [u for u in adj[v] if pos[u] < pos[v]]
            assert r.parent[v] == (max(earlier, key=lambda u: pos[u]) if earlier else -1)
        if not r.chordal:
            v, x, z = r.witness
            assert (v, x, z) == witness_by_definition(r.order.tolist(), adj)
            assert x == r.parent[v]
            assert is_chordless_cycle(r.cycle.tolist(), adj)
            assert r.cycle.tolist() == certificate_by_enumeration(n, adj, v, x, z)
            assert not r.fallback
    if n in CHORDAL_COUNTS_BY_HAND:
        assert count == CHORDAL_COUNTS_BY_HAND[n]


@pytest.mark.slow
def test_exhaustive_six():
    n = 6
    fallbacks = 0
    for mask, pairs, adj in all_graphs(n):
        g = graph_of(n, adj)
        r = oracle.chordal_test(g)
        assert r.order.tolist() == lexbfs_by_labels(n, adj), mask
        holes = chordal_by_holes(n, adj)
        assert r.chordal == holes, mask
        if not r.chordal:
            assert is_chordless_cycle(r.cycle.tolist(), adj)
            v, x, z = r.witness
            assert (v, x, z) == witness_by_definition(r.order.tolist(), adj)
            assert r.cycle.tolist() == certificate_by_enumeration(n, adj, v, x, z)
            fallbacks += r.fallback
    assert fallbacks == 0


# ---------------------------------------------------------------------------
# Random graphs: label-string LexBFS, Property LB / B, Theorem 5.1
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,p,seed", [(12, 0.3, 1), (20, 0.15, 2), (30, 0.5, 3), (60, 0.05, 4), (80, 0.1, 5),
                                      (120, 0.03, 6), (200, 0.02, 7), (200, 0.3, 8)])
def test_random_vs_label_definition(n, p, seed):
    rng = np.random.default_rng(seed)
    adj = random_adj(n, p, rng)
    g = graph_of(n, adj)
    r = oracle.lexbfs(g)
    assert r.order.tolist() == lexbfs_by_labels(n, adj)
    if n <= 40:
        assert satisfies_lb(r.order.tolist(), adj)
        assert satisfies_b(r.order.tolist(), adj)
    else:
        assert satisfies_lb_fast(r.order, adj_matrix(n, adj))


@pytest.mark.parametrize("seed", range(6))
def test_relabelled_graphs_vs_label_definition(seed):
    # same graph, random vertex names: the order changes with the names but
    # always matches the definition
    g0 = gg.subtree(90, 25, 6, gg.graph_seed(77, seed))
    perm = gg.permutation(g0.n, seed + 1)
    g = gg.relabel(g0, perm)
    adj = g.adj_sets()
    r = oracle.chordal_test(g)
    assert r.order.tolist() == lexbfs_by_labels(g.n, adj)
    assert r.chordal


def test_lb_checker_rejects_non_lexbfs_order():
    # the LB checker itself must be able to say no: on P4 0-1-2-3 the order
    # 1,0,3,2 is not a BFS order (3 comes before 2 but only 2 is adjacent to 1)
    adj = [{1}, {0, 2}, {1, 3}, {2}]
    assert not satisfies_b([1, 0, 3, 2], adj)
    assert not satisfies_lb([1, 0, 3, 2], adj)
    assert satisfies_lb([1, 0, 2, 3], adj)


@pytest.mark.parametrize("n,p,seed", [(40, 0.2, 11), (100, 0.05, 12), (300, 0.01, 13), (500, 0.5, 14),
                                      (2000, 0.003, 15)])
def test_parent_test_equals_full_peo_test(n, p, seed):
    # Section 5.3: the parent-only test returns true iff every left
    # neighbourhood is a clique
    rng = np.random.default_rng(seed)
    A = np.triu(rng.random((n, n)) < p, 1)
    A = A | A.T
    g = gg.from_adjacency(A.astype(np.uint8))
    order = oracle.lexbfs(g).order
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    full = True
    first_bad = None
    for v in order:
        ln = np.nonzero(A[v] & (pos < pos[v]))[0]
        sub = A[np.ix_(ln, ln)] | np.eye(len(ln), dtype=bool)
        if not sub.all():
            full = False
            first_bad = int(v)
            break
    pr = oracle.peo(g, pos.astype(np.int32))
    assert pr.is_peo == full
    if not full:
        assert pr.witness[0] == first_bad


def test_peo_on_non_lexbfs_orders():
    # the test is defined for any order: the identity order on C4 0-1-2-3
    # fails at 3 (LN {0, 2}, p = 2, 0 not adjacent to 2)
    g = gg.from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)])
    pr = oracle.peo(g, np.arange(4, dtype=np.int32))
    assert not pr.is_peo and pr.witness == (3, 2, 0)
    # reversed order on a path is a PEO
    P = gg.from_edges(5, [(i, i + 1) for i in range(4)])
    assert oracle.peo(P, np.arange(5)[::-1].astype(np.int32).copy()).is_peo


# ---------------------------------------------------------------------------
# Families with known verdicts
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_families(seed):
    s = gg.graph_seed(1234, seed)
    # random recursive tree, subtree graph, disjoint cliques, split graph,
    # clique: all chordal
    rng = np.random.default_rng(seed)
    tree = gg.from_edges(400, [(int(rng.integers(0, i)), i) for i in range(1, 400)])
    for g in [tree, gg.subtree(300, 64, 8, s), gg.subtree(500, 500, 1, s), gg.split(20, 200, 7, s),
              gg.from_edges(30, list(itertools.combinations(range(30), 2)))]:
        r = oracle.chordal_test(g)
        assert r.chordal, g.name
        assert is_peo_full(r.order.tolist(), g.adj_sets())
    for L in (4, 5, 9, 12):
        h = gg.plant_subtree(200 + L, L, 50, 8, s, s + 1)
        r = oracle.chordal_test(h)
        assert not r.chordal
        assert is_chordless_cycle(r.cycle.tolist(), h.adj_sets())
        assert not r.fallback
    g, h = gg.split_pair(30, 100, 5, s)
    assert oracle.chordal_test(g).chordal
    r = oracle.chordal_test(h)
    assert not r.chordal and len(r.cycle) == 4 and is_chordless_cycle(r.cycle.tolist(), h.adj_sets())


def test_forced_fallback_gives_a_hole():
    for n in (4, 5, 8):
        g = gg.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
        r = oracle.chordal_test(g)
        cyc, fb = oracle.certificate(g, r.order, r.rank, r.witness, force_fallback=True)
        assert fb and is_chordless_cycle(cyc.tolist(), g.adj_sets())
    rng = np.random.default_rng(5)
    for _ in range(30):
        adj = random_adj(9, 0.35, rng)
        g = graph_of(9, adj)
        r = oracle.chordal_test(g)
        if r.chordal:
            continue
        cyc, fb = oracle.certificate(g, r.order, r.rank, r.witness, force_fallback=True)
        assert fb and is_chordless_cycle(cyc.tolist(), adj)


def test_empty_and_single():
    r = oracle.chordal_test(gg.from_edges(0, []))
    assert r.chordal and r.order.size == 0
    r = oracle.chordal_test(gg.from_edges(1, []))
    assert r.chordal and r.order.tolist() == [0] and r.parent.tolist() == [-1]


@pytest.mark.parametrize("cfg", ["small"])
def test_workload_verdicts(cfg):
    g, h = gg.config_single_small()
    rg, rh = oracle.chordal_test(g), oracle.chordal_test(h)
    assert rg.chordal and not rh.chordal
    assert is_chordless_cycle(rh.cycle.tolist(), h.adj_sets())
    # the planted 5-cycle lives on ids 1024..1028
    assert set(rh.cycle.tolist()) == set(range(1024, 1029))


@pytest.mark.parametrize("n,p,seed", [(7, 0.4, 21), (9, 0.35, 22), (12, 0.3, 23), (16, 0.25, 24), (25, 0.2, 25)])
def test_random_non_chordal_witness_and_certificate(n, p, seed):
    rng = np.random.default_rng(seed)
    seen = 0
    for _ in range(60):
        adj = random_adj(n, p, rng)
        g = graph_of(n, adj)
        r = oracle.chordal_test(g)
        assert r.chordal == chordal_by_elimination(n, adj)
        if r.chordal:
            continue
        seen += 1
        v, x, z = r.witness
        assert (v, x, z) == witness_by_definition(r.order.tolist(), adj)
        assert is_chordless_cycle(r.cycle.tolist(), adj)
        if n <= 16:
            assert r.cycle.tolist() == certificate_by_enumeration(n, adj, v, x, z)
        assert not r.fallback
    assert seen > 0


def test_bitset_from_csr_matches_the_generators_and_a_hand_example():
    """The oracle's bitset (rebuilt from the CSR) equals the generators' own
    bitset (built directly, the CSR derived from it), and a 70-vertex hand
    example crossing a word boundary."""
    import oracle as orc

    for g in (gg.gnp(300, 0.05, 3), gg.subtree(200, 50, 6, 4), gg.from_edges(130, [(0, 129), (64, 65), (63, 64)])):
        b = orc.bitset_from_csr(g.n, g.row_ptr, g.col_idx, g.W)
        assert np.array_equal(b, g.bits.reshape(g.n, g.W)), g.name
    b = orc.bitset_from_csr(70, np.array([0, 1] + [1] * 68 + [2], dtype=np.int32), np.array([69, 0], dtype=np.int32), 2)
    assert b[0, 1] == np.uint64(1 << 5) and b[69, 0] == np.uint64(1) and int(b.sum()) == (1 << 5) + 1


def test_bitset_from_csr_rejects_what_is_no_graph():
    """Ids outside 0..n-1 (even inside the row's padding words) and broken
    row pointers describe no graph on n vertices: rejected, not dropped."""
    import oracle as orc

    rp = np.array([0, 1, 2], dtype=np.int32)
    with pytest.raises(ValueError):
        orc.bitset_from_csr(2, rp, np.array([1, 2], dtype=np.int32), 1)     # id n, inside the word
    with pytest.raises(ValueError):
        orc.bitset_from_csr(2, rp, np.array([1, 64], dtype=np.int32), 2)    # id in a padding word
    with pytest.raises(ValueError):
        orc.bitset_from_csr(2, rp, np.array([1, -1], dtype=np.int32), 1)    # negative id
    with pytest.raises(ValueError):
        orc.bitset_from_csr(2, np.array([0, 2, 1], dtype=np.int32), np.array([1, 0], dtype=np.int32), 1)
    with pytest.raises(ValueError):
        orc.bitset_from_csr(70, np.zeros(71, dtype=np.int32), np.zeros(0, dtype=np.int32), 1)  # W too small
