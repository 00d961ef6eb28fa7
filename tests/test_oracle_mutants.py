"""Plant plausible mistakes in a copy of the oracle source (CPU only) and
check that the pins catch every one of them."""
import os
import subprocess
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from brute import (all_graphs, random_adj, witness_by_definition, certificate_by_enumeration, chordal_by_holes, is_chordless_cycle, lexbfs_by_labels, mcs_by_counts)
from conftest import load_golden

TESTS = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(TESTS)
SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, original text, mutated text): each is one plausible slip
MUTANTS = [
    ("new class after C (label order inverted)",
     "K[Cp].next = C;\n                K[Cp].prev = K[C].prev;\n                if (K[C].prev >= 0) K[K[C].prev].next = Cp; else first = Cp;\n                K[C].prev = Cp;",
     "K[Cp].prev = C;\n                K[Cp].next = K[C].next;\n                if (K[C].next >= 0) K[K[C].next].prev = Cp;\n                K[C].next = Cp;"),
    ("pivot = tail of the first class (largest-id tie-break)",
     "int x = K[c0].head;", "int x = K[c0].tail >= 0 ? K[c0].tail : K[c0].head;"),
    ("p(v) = earliest instead of latest earlier neighbour",
     "(best < 0 || rank[y] > rank[best])", "(best < 0 || rank[y] < rank[best])"),
    ("parent test keeps p itself in LN(v)",
     "if (rank[z] < rank[y] && z != x && mark[z] != x)", "if (rank[z] < rank[y] && mark[z] != x)"),
    ("witness z* of largest rank",
     "if (!found && (zs < 0 || rank[z] < rank[zs])) zs = z;", "if (!found && (zs < 0 || rank[z] > rank[zs])) zs = z;"),
    ("certificate predecessor of largest id",
     "if (level[u] == l - 1) { pred = u; break; }", "if (level[u] == l - 1) { pred = u; }"),
    ("certificate path allowed through N(v*)",
     "inA[c] = 0;\n    for (int j = row_ptr[c]; j < row_ptr[c + 1]; j++) inA[col_idx[j]] = 0;", "inA[c] = 0;"),
    ("MCS raises the pivot's label (the box's literal text)",
     "label[y] += 1;\n            parent[y] = x;\n            mcs_entry e = {label[y], y};",
     "label[x] += 1;\n            parent[y] = x;\n            mcs_entry e = {label[y], y};"),
    ("MCS ties to the largest id",
     "return a.label > b.label || (a.label == b.label && a.id < b.id);",
     "return a.label > b.label || (a.label == b.label && a.id > b.id);"),
    ("MCS parent = first adjacent pivot",
     "            parent[y] = x;\n            mcs_entry e = {label[y], y};",
     "            if (parent[y] < 0) parent[y] = x;\n            mcs_entry e = {label[y], y};"),
]


def run_pins():
    """A fast subset of the pins; returns a list of failure descriptions."""
    fails = []
    for name in ("c4.txt", "c5.txt", "two_triangles.txt"):
        ex = load_golden(name)
        g = gg.from_edges(ex["n"], ex["edges"])
        try:
            r = oracle.chordal_test(g)
        except RuntimeError as e:
            fails.append(f"{name}: {e}")
            continue
        if (r.order.tolist() != ex["order"] or r.parent.tolist() != ex["parent"] or r.chordal != ex["chordal"]
                or list(r.witness) != ex["witness"] or r.cycle.tolist() != ex["cycle"]):
            fails.append(name)
    for n in (4, 5):
        for mask, pairs, adj in all_graphs(n):
            g = gg.from_edges(n, [(a, b) for a in range(n) for b in adj[a] if a < b])
            try:
                r = oracle.chordal_test(g)
            except RuntimeError as e:
                fails.append(f"n={n} mask={mask}: {e}")
                break
            if r.order.tolist() != lexbfs_by_labels(n, adj) or r.chordal != chordal_by_holes(n, adj):
                fails.append(f"n={n} mask={mask}")
                break
            if not r.chordal:
                v, x, z = r.witness
                if (not is_chordless_cycle(r.cycle.tolist(), adj)
                        or r.cycle.tolist() != certificate_by_enumeration(n, adj, v, x, z)):
                    fails.append(f"cert n={n} mask={mask}")
                    break
    for n in (4, 5):
        for mask, pairs, adj in all_graphs(n):
            g = gg.from_edges(n, [(a, b) for a in range(n) for b in adj[a] if a < b])
            try:
                r = oracle.chordal_test(g, "mcs")
            except RuntimeError as e:
                fails.append(f"mcs n={n} mask={mask}: {e}")
                break
            if r.order.tolist() != mcs_by_counts(n, adj) or r.chordal != chordal_by_holes(n, adj):
                fails.append(f"mcs n={n} mask={mask}")
                break
            if not r.chordal and tuple(r.witness) != witness_by_definition(r.order.tolist(), adj):
                fails.append(f"mcs witness n={n} mask={mask}")
                break
            m = oracle.mcs(g)
            latest = [max((u for u in adj[v] if m.rank[u] < m.rank[v]), key=lambda u: m.rank[u], default=-1)
                      for v in range(n)]
            if m.parent.tolist() != latest:
                fails.append(f"mcs parent n={n} mask={mask}")
                break
    rng = np.random.default_rng(31)
    for trial in range(80):
        n = 8 + trial % 5
        adj = random_adj(n, 0.35, rng)
        g = gg.from_edges(n, [(a, b) for a in range(n) for b in adj[a] if a < b])
        try:
            r = oracle.chordal_test(g)
        except RuntimeError as e:
            fails.append(f"random {trial}: {e}")
            break
        if r.chordal != chordal_by_holes(n, adj):
            fails.append(f"random {trial} verdict")
            break
        if not r.chordal and tuple(r.witness) != witness_by_definition(r.order.tolist(), adj):
            fails.append(f"random {trial} witness")
            break
    return fails


def test_unmutated_copy_passes(tmp_path):
    so = str(tmp_path / "liboracle_copy.so")
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", so, SRC])
    with oracle.use_library(so):
        assert run_pins() == []


@pytest.mark.parametrize("idx", range(len(MUTANTS)))
def test_mutant_is_caught(tmp_path, idx):
    # A mutant may also crash on inputs its own mistake makes inconsistent;
    # it runs in a child process, and a crash counts as caught.
    name, old, new = MUTANTS[idx]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not found: {name}"
    path = tmp_path / "oracle_mut.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "liboracle_mut.so")
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", so, str(path)])
    code = ("import sys; sys.path[:0] = [%r, %r]\n"
            "import oracle, test_oracle_mutants as t\n"
            "with oracle.use_library(%r):\n"
            "    sys.exit(1 if t.run_pins() else 0)\n") % (ROOT, TESTS, so)
    proc = subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=300)
    assert proc.returncode != 0, f"pins did not catch: {name}"


# Planted mistakes in the Python part of the oracle (multi-sweep LexBFS+ and
# the unit interval test), each in a copy of the package run in a child
# process against the interval pins.
PY_MUTANTS = [
    ("LexBFS+ ties to the first instead of the last vertex of the previous order",
     "    new_id = n - 1 - pos\n", "    new_id = pos.copy()\n"),
    ("open instead of closed neighbourhoods",
     "        ps = np.concatenate([pos[nbrs], [i]])\n", "        ps = pos[nbrs] if len(nbrs) else np.array([i])\n"),
    ("two sweeps instead of three",
     "    s3 = lexbfs_plus(g, s2).order\n", "    s3 = s2\n"),
    ("witness b = the latest instead of the earliest non-member of the span",
     "        b_pos = lo + int(np.argmin(inside))\n",
     "        b_pos = hi - int(np.argmin(inside[::-1]))\n"),
    ("witness triple forms swapped",
     "        if b_pos < i:\n", "        if b_pos > i:\n"),
    ("witness orientation by the middle of the span instead of by v",
     "        if b_pos < i:\n", "        if 2 * b_pos < lo + hi:\n"),
]


@pytest.mark.parametrize("idx", range(len(PY_MUTANTS)))
def test_python_mutant_is_caught(tmp_path, idx):
    import shutil

    name, old, new = PY_MUTANTS[idx]
    pkg = os.path.dirname(oracle.__file__)
    dst = tmp_path / "oracle"
    shutil.copytree(pkg, dst, ignore=shutil.ignore_patterns("__pycache__"))
    src = (dst / "__init__.py").read_text()
    assert src.count(old) == 1, f"mutation site not found: {name}"
    (dst / "__init__.py").write_text(src.replace(old, new))
    code = ("import sys; sys.path[:0] = [%r, %r, %r]\n"
            "import oracle\n"
            "assert oracle.__file__.startswith(%r)\n"
            "import test_oracle_interval as t, pytest\n"
            "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', t.__file__]))\n") % (
        str(tmp_path), ROOT, TESTS, str(tmp_path))
    proc = subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=600, cwd=str(tmp_path))
    assert proc.returncode != 0, f"pins did not catch: {name}"


def test_python_unmutated_copy_passes(tmp_path):
    import shutil

    pkg = os.path.dirname(oracle.__file__)
    shutil.copytree(pkg, tmp_path / "oracle", ignore=shutil.ignore_patterns("__pycache__"))
    code = ("import sys; sys.path[:0] = [%r, %r, %r]\n"
            "import oracle\n"
            "assert oracle.__file__.startswith(%r)\n"
            "import test_oracle_interval as t, pytest\n"
            "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', t.__file__]))\n") % (
        str(tmp_path), ROOT, TESTS, str(tmp_path))
    proc = subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=600, cwd=str(tmp_path))
    assert proc.returncode == 0, proc.stdout.decode()[-2000:] + proc.stderr.decode()[-2000:]
