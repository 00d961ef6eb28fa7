"""Brute-force checkers written from definitions, used to pin the oracle.

Nothing here calls the oracle or the GPU library. Graphs are given as a list
of neighbour sets ``adj`` over vertices 0..n-1.

* :func:`lexbfs_by_labels` -- the label-string LexBFS of Section 4.1 taken
  literally: labels are Python lists, the largest label (lexicographic, a
  proper prefix is smaller) is numbered next, smallest id on ties, and step i
  (1-based) appends n - i to the label of every unnumbered neighbour.
* :func:`satisfies_lb` -- Property LB (Lemma 4.2): for positions a < b < c with
  ac an edge and ab not, some d < a has db an edge and dc not.
* :func:`satisfies_b` -- Property B (Lemma 4.1).
* :func:`chordal_by_holes` -- the definition of chordality (Section 3.1):
  no induced cycle of length >= 4, by subset enumeration.
* :func:`chordal_by_elimination` -- greedy removal of simplicial vertices.
* :func:`is_peo_full` -- every left neighbourhood induces a clique (the
  perfect-elimination definition of Section 3.1).
* :func:`certificate_by_enumeration` -- all shortest x*-z* paths avoiding
  N[v*] enumerated explicitly, the one whose reversed vertex sequence is
  lexicographically smallest selected.
* :func:`is_chordless_cycle` -- validity of a certificate.
* :func:`parents_by_definition` -- p(v), the latest earlier neighbour.
* :func:`three_sweeps_by_labels`, :func:`unit_interval_witness_by_definition`
  -- the third order of the unit interval test from three label-string
  sweeps, and its witness rule written out step by step.
"""
from __future__ import annotations

import itertools
from typing import List, Optional, Sequence, Set

import numpy as np


def lexbfs_by_labels(n: int, adj: Sequence[Set[int]]) -> List[int]:
    label = [[] for _ in range(n)]
    numbered = [False] * n
    order = []
    for i in range(1, n + 1):
        best = None
        for v in range(n):
            if numbered[v]:
                continue
            if best is None or label[v] > label[best]:
                best = v
        x = best
        numbered[x] = True
        order.append(x)
        for y in adj[x]:
            if not numbered[y]:
                label[y] = label[y] + [n - i]
    return order


def lexbfs_plus_by_labels(n: int, adj: Sequence[Set[int]], prev: Sequence[int]) -> List[int]:
    """LexBFS with literal label strings, ties to the vertex that comes last
    in the previous order `prev` (the '+' rule)."""
    pos = {v: i for i, v in enumerate(prev)}
    label = [[] for _ in range(n)]
    numbered = [False] * n
    order = []
    for i in range(1, n + 1):
        best = None
        for v in range(n):
            if numbered[v]:
                continue
            if best is None or label[v] > label[best] or (label[v] == label[best] and pos[v] > pos[best]):
                best = v
        numbered[best] = True
        order.append(best)
        for y in adj[best]:
            if not numbered[y]:
                label[y] = label[y] + [n - i]
    return order


def parents_by_definition(order: Sequence[int], adj: Sequence[Set[int]]) -> List[int]:
    """p(v) of Section 5.2 for every vertex: the neighbour of v that comes
    latest among those before v in `order`, or -1."""
    pos = {v: i for i, v in enumerate(order)}
    par = [-1] * len(order)
    for v in order:
        earlier = [u for u in adj[v] if pos[u] < pos[v]]
        if earlier:
            par[v] = max(earlier, key=lambda u: pos[u])
    return par


def three_sweeps_by_labels(n: int, adj: Sequence[Set[int]]) -> List[int]:
    """The third order of the three-sweep unit interval test, every sweep
    taken with literal label strings: LexBFS (smallest id on ties), then
    LexBFS+ after it, then LexBFS+ after that."""
    s1 = lexbfs_by_labels(n, adj)
    s2 = lexbfs_plus_by_labels(n, adj, s1)
    return lexbfs_plus_by_labels(n, adj, s2)


def unit_interval_witness_by_definition(order: Sequence[int], adj: Sequence[Set[int]]):
    """The witness of a failed unit interval test, written out from its
    definition: walk the order from the front; the first vertex v whose
    closed neighbourhood does not occupy consecutive positions is the
    failing one. Its closed neighbourhood spans positions lo..hi; b is the
    vertex at the first position of that span that is neither v nor a
    neighbour of v. When b is placed before v the triple is
    (order[lo], b, v), otherwise (v, b, order[hi]). None if every closed
    neighbourhood is consecutive."""
    where = {}
    for i, v in enumerate(order):
        where[v] = i
    for i, v in enumerate(order):
        closed = set(adj[v])
        closed.add(v)
        spots = sorted(where[u] for u in closed)
        lo, hi = spots[0], spots[-1]
        if hi - lo + 1 == len(spots):
            continue
        b = None
        for j in range(lo, hi + 1):
            if order[j] not in closed:
                b = order[j]
                break
        if where[b] < i:
            return (order[lo], b, v)
        return (v, b, order[hi])
    return None


def closed_nbhds_consecutive(order: Sequence[int], adj: Sequence[Set[int]]) -> bool:
    pos = {v: i for i, v in enumerate(order)}
    for v in order:
        ps = [pos[u] for u in adj[v]] + [pos[v]]
        if max(ps) - min(ps) + 1 != len(ps):
            return False
    return True


def unit_interval_by_orderings(n: int, adj: Sequence[Set[int]]) -> bool:
    """Unit (proper) interval graph iff some vertex order makes every closed
    neighbourhood consecutive (Roberts); tried over all orders."""
    return any(closed_nbhds_consecutive(p, adj) for p in itertools.permutations(range(n)))


def has_induced_claw(n: int, adj: Sequence[Set[int]]) -> bool:
    for c in range(n):
        nb = sorted(adj[c])
        for a, b, d in itertools.combinations(nb, 3):
            if b not in adj[a] and d not in adj[a] and d not in adj[b]:
                return True
    return False


def mcs_by_counts(n: int, adj: Sequence[Set[int]]) -> List[int]:
    """Maximum Cardinality Search straight from its definition: every step
    recounts, for each unnumbered vertex, its numbered neighbours and takes
    the largest count (smallest id on ties)."""
    numbered = [False] * n
    order = []
    for _ in range(n):
        best, best_cnt = None, -1
        for v in range(n):
            if numbered[v]:
                continue
            cnt = sum(1 for u in adj[v] if numbered[u])
            if cnt > best_cnt:
                best, best_cnt = v, cnt
        numbered[best] = True
        order.append(best)
    return order


def satisfies_lb(order: Sequence[int], adj: Sequence[Set[int]]) -> bool:
    n = len(order)
    pos = {v: i for i, v in enumerate(order)}
    for ia in range(n):
        a = order[ia]
        for ib in range(ia + 1, n):
            b = order[ib]
            if b in adj[a]:
                continue
            for ic in range(ib + 1, n):
                c = order[ic]
                if c not in adj[a]:
                    continue
                if not any((b in adj[order[d]]) and (c not in adj[order[d]]) for d in range(ia)):
                    return False
    return True


def satisfies_lb_fast(order: np.ndarray, A: np.ndarray) -> bool:
    """Property LB with numpy boolean matrices, for n up to a few hundred.

    A is the 0/1 adjacency matrix in vertex ids. Re-index by position so
    that "d < a" is a prefix. For every pair (a, b) with a < b, ab not an
    edge, the set of c > b adjacent to a must be covered by
    union_{d < a, db edge} (not N(d)), i.e. no c > b with ac edge and dc
    edge for every d < a adjacent to b.
    """
    P = A[np.ix_(order, order)].astype(bool)
    n = P.shape[0]
    for a in range(n):
        left = P[:a]                      # rows d < a
        for b in range(a + 1, n):
            if P[a, b]:
                continue
            cs = np.nonzero(P[a, b + 1:])[0] + b + 1
            if cs.size == 0:
                continue
            ds = np.nonzero(left[:, b])[0]
            if ds.size == 0:
                return False
            # each c needs some d with dc not an edge
            covered = (~left[np.ix_(ds, cs)]).any(axis=0)
            if not covered.all():
                return False
    return True


def satisfies_b(order: Sequence[int], adj: Sequence[Set[int]]) -> bool:
    n = len(order)
    for ia in range(n):
        a = order[ia]
        for ib in range(ia + 1, n):
            b = order[ib]
            if b in adj[a]:
                continue
            for ic in range(ib + 1, n):
                c = order[ic]
                if c in adj[a] and not any(b in adj[order[d]] for d in range(ia)):
                    return False
    return True


def _is_cycle(sub: Sequence[int], adj: Sequence[Set[int]]) -> bool:
    s = set(sub)
    for v in sub:
        if len(adj[v] & s) != 2:
            return False
    # connected?
    start = sub[0]
    seen = {start}
    stack = [start]
    while stack:
        u = stack.pop()
        for w in adj[u] & s:
            if w not in seen:
                seen.add(w)
                stack.append(w)
    return len(seen) == len(s)


def chordal_by_holes(n: int, adj: Sequence[Set[int]]) -> bool:
    for k in range(4, n + 1):
        for sub in itertools.combinations(range(n), k):
            if _is_cycle(sub, adj):
                return False
    return True


def chordal_by_elimination(n: int, adj: Sequence[Set[int]]) -> bool:
    alive = set(range(n))
    while alive:
        for v in sorted(alive):
            nb = adj[v] & alive
            if all(b in adj[a] for a, b in itertools.combinations(sorted(nb), 2)):
                alive.remove(v)
                break
        else:
            return False
    return True


def is_peo_full(order: Sequence[int], adj: Sequence[Set[int]]) -> bool:
    pos = {v: i for i, v in enumerate(order)}
    for v in order:
        ln = [u for u in adj[v] if pos[u] < pos[v]]
        for a, b in itertools.combinations(ln, 2):
            if b not in adj[a]:
                return False
    return True


def first_non_simplicial(order: Sequence[int], adj: Sequence[Set[int]]) -> Optional[int]:
    pos = {v: i for i, v in enumerate(order)}
    for v in order:
        ln = [u for u in adj[v] if pos[u] < pos[v]]
        if any(b not in adj[a] for a, b in itertools.combinations(ln, 2)):
            return v
    return None


def witness_by_definition(order: Sequence[int], adj: Sequence[Set[int]]):
    """(v*, x*, z*): v* the first vertex of the order whose left
    neighbourhood is not a clique, x* its latest earlier neighbour, z* the
    earliest earlier neighbour of v* other than x* and not adjacent to x*."""
    v = first_non_simplicial(order, adj)
    if v is None:
        return (-1, -1, -1)
    pos = {u: i for i, u in enumerate(order)}
    ln = sorted((u for u in adj[v] if pos[u] < pos[v]), key=lambda u: pos[u])
    x = ln[-1]
    z = next(u for u in ln if u != x and u not in adj[x])
    return (v, x, z)


def is_chordless_cycle(cycle: Sequence[int], adj: Sequence[Set[int]]) -> bool:
    L = len(cycle)
    if L < 4 or len(set(cycle)) != L:
        return False
    for i in range(L):
        for j in range(i + 1, L):
            consecutive = (j == i + 1) or (i == 0 and j == L - 1)
            if (cycle[j] in adj[cycle[i]]) != consecutive:
                return False
    return True


def certificate_by_enumeration(n: int, adj: Sequence[Set[int]], v: int, x: int, z: int) -> Optional[List[int]]:
    """[v, x, ..., z] for the shortest x-z paths inside (V minus N[v]) plus
    {x, z}, choosing the path whose sequence read from z backwards is
    lexicographically smallest. Exhaustive over simple paths (tiny n)."""
    allowed = (set(range(n)) - adj[v] - {v}) | {x, z}
    best: Optional[List[int]] = None

    def dfs(path: List[int], seen: Set[int]):
        nonlocal best
        u = path[-1]
        if best is not None and len(path) > len(best):
            return
        if u == z:
            if best is None or len(path) < len(best) or (len(path) == len(best) and path[::-1] < best[::-1]):
                best = list(path)
            return
        for w in sorted(adj[u]):
            if w in allowed and w not in seen:
                seen.add(w)
                path.append(w)
                dfs(path, seen)
                path.pop()
                seen.remove(w)

    dfs([x], {x})
    if best is None:
        return None
    return [v] + best


def all_graphs(n: int):
    """Every labelled simple graph on n vertices, as neighbour-set lists."""
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        adj = [set() for _ in range(n)]
        for k, (a, b) in enumerate(pairs):
            if (mask >> k) & 1:
                adj[a].add(b)
                adj[b].add(a)
        yield mask, pairs, adj


def random_adj(n: int, p: float, rng: np.random.Generator) -> List[Set[int]]:
    M = np.triu(rng.random((n, n)) < p, 1)
    adj = [set() for _ in range(n)]
    for a, b in zip(*np.nonzero(M)):
        adj[int(a)].add(int(b))
        adj[int(b)].add(int(a))
    return adj


def adj_matrix(n: int, adj: Sequence[Set[int]]) -> np.ndarray:
    A = np.zeros((n, n), dtype=bool)
    for v in range(n):
        for u in adj[v]:
            A[v, u] = True
    return A
