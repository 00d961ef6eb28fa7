"""GPU parity: the HIP path through the C ABI against the CPU oracle,
element by element (orders, ranks, parents, verdicts, witnesses and
certificates are integers: the bar is bit-exact)."""
import itertools
import os
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1508_06329_amd as lx  # noqa: E402

DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check_single(g, flags=0, tag=""):
    say(f"[parity] {tag} {g.name} n={g.n} m={g.m} flags={flags}")
    ref = oracle.chordal_test(g)
    dg = lx.DeviceGraph.from_host(g, DEV)
    r = lx.chordal_test(dg, flags=flags)
    assert np.array_equal(r.order.cpu().numpy(), ref.order), "order"
    assert np.array_equal(r.rank.cpu().numpy(), ref.rank), "rank"
    assert np.array_equal(r.parent.cpu().numpy(), ref.parent), "parent"
    assert r.chordal == ref.chordal
    if flags & lx.LEXBFS_FLAG_FORCE_FALLBACK and not ref.chordal:
        cyc, fb = oracle.certificate(g, ref.order, ref.rank, ref.witness, force_fallback=True)
        assert r.fallback and fb
        assert r.witness == ref.witness
        assert r.cycle_list == cyc.tolist()
    else:
        assert r.witness == ref.witness
        assert r.cycle_list == ref.cycle.tolist()
        assert r.fallback == ref.fallback
    return r, ref


# ---------------------------------------------------------------------------
# Small and structured graphs
# ---------------------------------------------------------------------------

def structured_cases():
    cases = []
    for n in (0, 1, 2, 3, 5, 63, 64, 65, 127, 129, 1000):
        cases.append(gg.from_edges(n, list(itertools.combinations(range(n), 2)) if n <= 300 else [], f"K{n}"))
        cases.append(gg.from_edges(n, [], f"E{n}"))
        cases.append(gg.from_edges(n, [(i, i + 1) for i in range(n - 1)], f"P{n}"))
        if n >= 4:
            cases.append(gg.from_edges(n, [(i, (i + 1) % n) for i in range(n)], f"C{n}"))
        if n >= 3:
            cases.append(gg.from_edges(n, [(n // 2, v) for v in range(n) if v != n // 2], f"S{n}"))
    from conftest import load_golden
    for name in ("c4.txt", "c5.txt", "two_triangles.txt"):
        ex = load_golden(name)
        cases.append(gg.from_edges(ex["n"], ex["edges"], name))
    return cases


@pytest.mark.parametrize("idx", range(len(structured_cases())))
def test_structured(idx):
    g = structured_cases()[idx]
    check_single(g, tag=f"structured[{idx}]")


@pytest.mark.parametrize("n,p,seed", [(10, 0.4, 1), (50, 0.2, 2), (64, 0.5, 3), (100, 0.05, 4), (300, 0.02, 5),
                                      (700, 0.3, 6), (1500, 0.004, 7), (4097, 0.002, 8), (5000, 0.3, 9),
                                      (9000, 0.001, 10)])
def test_random_gnp(n, p, seed):
    check_single(gg.gnp(n, p, seed), tag="gnp")


@pytest.mark.parametrize("n,T,s,seed", [(100, 30, 5, 1), (1024, 256, 8, 2), (3000, 700, 10, 3), (8000, 2000, 12, 4)])
def test_random_subtree(n, T, s, seed):
    g = gg.subtree(n, T, s, seed)
    check_single(g, tag="subtree")
    h = gg.plant(g, 4 + seed, seed + 100)
    check_single(h, tag="planted")


@pytest.mark.parametrize("K,I,a", [(20, 100, 5), (200, 2000, 16)])
def test_split_pairs(K, I, a):
    for g in gg.split_pair(K, I, a, 7):
        check_single(g, tag="split")


@pytest.mark.parametrize("seed", range(3))
def test_forced_fallback(seed):
    g = gg.gnp(200, 0.03, 50 + seed)
    check_single(g, flags=lx.LEXBFS_FLAG_FORCE_FALLBACK, tag="fallback")
    h = gg.plant(gg.subtree(300, 80, 6, seed), 6, seed)
    check_single(h, flags=lx.LEXBFS_FLAG_FORCE_FALLBACK, tag="fallback")


# ---------------------------------------------------------------------------
# Full-size single-graph workloads
# ---------------------------------------------------------------------------

def test_workload_small_full():
    for g in gg.config_single_small():
        check_single(g, tag="N=1024 workload")


def test_workload_large_sparse_full():
    for g in gg.config_single_large():
        check_single(g, tag="N=16384 workload")


def test_workload_split_65536_full():
    for g in gg.config_worst_steps():
        r, ref = check_single(g, tag="N=65536 split workload")
    assert not ref.chordal and len(ref.cycle) == 4


# Split graphs at n = 65,536 (1,024-lane team, class tables in L2) whose
# pivots have thousands of neighbours spread over every lane from the first
# step on: the clique's vertices hold the next pivot at every clique step,
# so a lost or wrong contribution of their lane to a selection shows at once.
def heavy_split(K):
    return gg.split(K, 65536 - K, min(64, max(1, K // 2)), 1000 + K)


def moved_clique(base):
    """The 32-clique split graph with ids [0, 64) and [base, base + 64)
    swapped: the clique sits on another lane and wave."""
    g = heavy_split(32)
    perm = np.arange(g.n, dtype=np.int64)
    perm[0:64] = np.arange(base, base + 64)
    perm[base:base + 64] = np.arange(64)
    return gg.relabel(g, perm)


@pytest.mark.parametrize("K", [16, 32, 128, 512, 2048])
def test_split_heavy_steps_65536(K):
    check_single(heavy_split(K), tag=f"heavy split, clique of {K}")


@pytest.mark.parametrize("base", [64, 20480, 21568])
def test_split_heavy_steps_clique_on_other_lanes(base):
    check_single(moved_clique(base), tag=f"heavy split, clique at {base}")


HEAVY_SMALLER = [(1024, 16), (1024, 64), (4096, 16), (4096, 256), (16384, 64), (16384, 256), (32768, 16),
                 (32768, 256)]


def heavy_split_n(n, K):
    return gg.split(K, n - K, min(64, max(1, K // 2)), 7000 + K + n)


@pytest.mark.parametrize("n,K", HEAVY_SMALLER)
def test_split_heavy_steps_smaller_teams(n, K):
    """The same heavy steps on the 128-, 256- and 512-lane teams (LDS class
    tables, compact layout at n = 32,768)."""
    check_single(heavy_split_n(n, K), tag=f"heavy split n={n}, clique of {K}")


@pytest.mark.parametrize("n,K", [(65536, 32), (16384, 64)])
def test_split_heavy_steps_mcs_and_per_step(n, K):
    """The heavy split graphs through the MCS order (1,024- and 512-lane
    MCS kernels) and the per-step-launch form of LexBFS."""
    g = heavy_split(K) if n == 65536 else heavy_split_n(n, K)
    say(f"[parity] heavy split MCS n={n} K={K}")
    ref = oracle.chordal_test(g, "mcs")
    r = lx.chordal_test(lx.DeviceGraph.from_host(g, DEV), flags=lx.LEXBFS_FLAG_MCS)
    assert np.array_equal(r.order.cpu().numpy(), ref.order), "MCS order"
    assert np.array_equal(r.parent.cpu().numpy(), ref.parent), "MCS parent"
    assert r.chordal == ref.chordal and r.witness == ref.witness and r.cycle_list == ref.cycle.tolist()
    check_single(g, flags=lx.LEXBFS_FLAG_PER_STEP, tag=f"heavy split per-step n={n} K={K}")


def test_batch_heavy_steps_every_tier():
    check_batch([heavy_split_n(n, K) for n, K in HEAVY_SMALLER], tag="heavy split graphs, n = 1,024 .. 32,768")


# ---------------------------------------------------------------------------
# lexbfs_order entry point, determinism
# ---------------------------------------------------------------------------

def test_lexbfs_order_entry_point():
    g = gg.subtree(2000, 500, 8, 11)
    ref = oracle.lexbfs(g)
    dg = lx.DeviceGraph.from_host(g, DEV)
    order, rank, parent = lx.lexbfs_order(dg)
    torch.cuda.synchronize()
    assert np.array_equal(order.cpu().numpy(), ref.order)
    assert np.array_equal(rank.cpu().numpy(), ref.rank)
    assert np.array_equal(parent.cpu().numpy(), ref.parent)


def test_repeat_is_deterministic():
    g = gg.gnp(3000, 0.01, 99)
    dg = lx.DeviceGraph.from_host(g, DEV)
    a = lx.chordal_test(dg)
    b = lx.chordal_test(dg, stream=torch.cuda.Stream())
    assert torch.equal(a.order, b.order) and a.witness == b.witness and a.cycle_list == b.cycle_list


# ---------------------------------------------------------------------------
# Batch
# ---------------------------------------------------------------------------

def check_batch(graphs, tuning=None, tag=""):
    say(f"[parity] batch {tag} count={len(graphs)} tuning={tuning}")
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    rs = lx.chordal_test_batch(dgs, outputs=True, tuning=tuning)
    for g, r in zip(graphs, rs):
        ref = oracle.chordal_test(g)
        assert np.array_equal(r.order.cpu().numpy(), ref.order), g.name
        assert np.array_equal(r.parent.cpu().numpy(), ref.parent), g.name
        assert r.chordal == ref.chordal and r.witness == ref.witness, g.name
        assert r.cycle_list == ref.cycle.tolist(), g.name
    return rs


def test_batch_mix_small():
    graphs = gg.config_batch(count=96, lo=32, hi=4096, seed=5)
    graphs += [gg.from_edges(0, []), gg.from_edges(1, []), gg.from_edges(5, [(i, (i + 1) % 5) for i in range(5)])]
    check_batch(graphs, tag="mix")
    check_batch(graphs, tuning={"wave_max_n": 256}, tag="mix")
    check_batch(graphs, tuning={"wave_max_n": 4096}, tag="mix")


def test_batch_equals_single():
    graphs = gg.config_batch(count=24, lo=32, hi=2000, seed=6)
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    rs = lx.chordal_test_batch(dgs, outputs=True)
    for dg, r in zip(dgs, rs):
        s = lx.chordal_test(dg)
        assert torch.equal(s.order, r.order) and s.witness == r.witness and s.cycle_list == r.cycle_list


def test_batch_workload_full():
    graphs = gg.config_batch()  # 4,096 graphs, N log-uniform on [32, 4096]
    say(f"[parity] batch workload full count={len(graphs)}")
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    rs = lx.chordal_test_batch(dgs, outputs=True)
    bad = []
    for i, (g, r) in enumerate(zip(graphs, rs)):
        ref = oracle.chordal_test(g)
        if not (np.array_equal(r.order.cpu().numpy(), ref.order) and np.array_equal(r.rank.cpu().numpy(), ref.rank)
                and np.array_equal(r.parent.cpu().numpy(), ref.parent) and r.chordal == ref.chordal
                and r.witness == ref.witness and r.cycle_list == ref.cycle.tolist() and r.fallback == ref.fallback):
            bad.append(i)
    assert bad == []
    assert sum(r.chordal for r in rs) == 2048


def test_batch_workload_full_mcs():
    """The whole 4,096-graph batch workload under LEXBFS_FLAG_MCS (the MCS
    order of Section 5.1 and the same test, Theorem 5.2): order, rank,
    parent, verdict, witness and certificate of every graph."""
    graphs = gg.config_batch()
    say(f"[parity] batch workload full MCS count={len(graphs)}")
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    rs = lx.chordal_test_batch(dgs, outputs=True, flags=lx.LEXBFS_FLAG_MCS)
    bad = []
    for i, (g, r) in enumerate(zip(graphs, rs)):
        ref = oracle.chordal_test(g, "mcs")
        if not (np.array_equal(r.order.cpu().numpy(), ref.order) and np.array_equal(r.rank.cpu().numpy(), ref.rank)
                and np.array_equal(r.parent.cpu().numpy(), ref.parent) and r.chordal == ref.chordal
                and r.witness == ref.witness and r.cycle_list == ref.cycle.tolist() and r.fallback == ref.fallback):
            bad.append(i)
    assert bad == []
    assert sum(r.chordal for r in rs) == 2048


# ---------------------------------------------------------------------------
# Sizes whose LexBFS state only fits LDS in the compact layout
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["gnp25000", "subtree32768_planted", "split30000", "edgeless20000"])
def test_compact_mode_sizes(case):
    if case == "gnp25000":
        g = gg.gnp(25000, 0.0004, 21)
    elif case == "subtree32768_planted":
        g = gg.plant(gg.subtree(32760, 8000, 12, 22), 8, 23)
    elif case == "split30000":
        g = gg.split_pair(1000, 29000, 12, 24)[1]
    else:
        g = gg.from_edges(20000, [])
    check_single(g, tag="compact")


# ---------------------------------------------------------------------------
# Batch schedules: autotuner, block-per-graph only, HIP graph replay
# ---------------------------------------------------------------------------

def test_block_per_graph_schedule():
    graphs = gg.config_batch(count=48, lo=32, hi=3000, seed=8)
    graphs.append(gg.from_edges(0, []))
    check_batch(graphs, tuning={"wave_max_n": -1}, tag="block per graph")


def test_autotuner_picks_a_valid_schedule():
    from paper_1508_06329_amd import autotune

    graphs = gg.config_batch(count=64, lo=32, hi=4096, seed=9)
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    out = autotune.autotune_batch(dgs, candidates=(-1, 256, 1024), reps=2)
    say(f"[parity] autotune table {out['ms']}")
    assert set(out["ms"]) == {-1, 256, 1024}
    best = out["tuning"]["wave_max_n"]
    assert out["ms"][best] == min(t for t in out["ms"].values() if t is not None)
    check_batch(graphs, tuning=out["tuning"], tag="autotuned")


def test_batch_plan_hip_graph_replay():
    graphs = gg.config_batch(count=40, lo=32, hi=2500, seed=10)
    refs = [oracle.chordal_test(g) for g in graphs]
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    plan = lx.BatchPlan(dgs, outputs=True)
    say("[parity] hip graph capture of a batch plan")
    graph = plan.capture()
    for rep in range(3):
        plan.res.fill_(-7)  # eager work between replays
        for t in plan.tens:
            t["order"].fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        rs = plan.results()
        for g, r, ref in zip(graphs, rs, refs):
            assert np.array_equal(r.order.cpu().numpy(), ref.order), (rep, g.name)
            assert r.chordal == ref.chordal and r.witness == ref.witness, (rep, g.name)
            assert r.cycle_list == ref.cycle.tolist(), (rep, g.name)
    plan.close()


# ---------------------------------------------------------------------------
# Per-step launch form of LexBFS (comparison path, LEXBFS_FLAG_PER_STEP)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("idx", [0, 1, 2, 3, 5, 9, 14, 20, 33, 40, 47])
def test_per_step_structured(idx):
    cases = structured_cases()
    g = cases[idx % len(cases)]
    check_single(g, flags=lx.LEXBFS_FLAG_PER_STEP, tag="per-step")


@pytest.mark.parametrize("seed", range(3))
def test_per_step_random(seed):
    check_single(gg.gnp(700, 0.01, 70 + seed), flags=lx.LEXBFS_FLAG_PER_STEP, tag="per-step")
    check_single(gg.plant(gg.subtree(900, 200, 8, seed), 6, seed), flags=lx.LEXBFS_FLAG_PER_STEP, tag="per-step")
    for g in gg.split_pair(30, 300, 6, 80 + seed):
        check_single(g, flags=lx.LEXBFS_FLAG_PER_STEP, tag="per-step")


def test_per_step_workload_small_full():
    for g in gg.config_single_small():
        check_single(g, flags=lx.LEXBFS_FLAG_PER_STEP, tag="per-step N=1024 workload")


def test_per_step_workload_split_65536_full():
    for g in gg.config_worst_steps():
        check_single(g, flags=lx.LEXBFS_FLAG_PER_STEP, tag="per-step N=65536 split workload")


def test_batch_forced_fallback_matches_single():
    graphs = [gg.gnp(150, 0.04, 90 + s) for s in range(4)] + [gg.plant(gg.subtree(2500, 600, 8, 5), 7, 5)]
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    rs = lx.chordal_test_batch(dgs, outputs=True, flags=lx.LEXBFS_FLAG_FORCE_FALLBACK)
    for g, dg, r in zip(graphs, dgs, rs):
        s = lx.chordal_test(dg, flags=lx.LEXBFS_FLAG_FORCE_FALLBACK)
        assert r.chordal == s.chordal and r.witness == s.witness, g.name
        assert r.cycle_list == s.cycle_list and r.fallback == s.fallback, g.name
        if not s.chordal:
            ref = oracle.chordal_test(g)
            cyc, fb = oracle.certificate(g, ref.order, ref.rank, ref.witness, force_fallback=True)
            assert r.cycle_list == cyc.tolist() and fb


def test_batch_size_limit():
    from paper_1508_06329_amd import _lib

    lim = int(_lib.load().lexbfs_batch_max_n())
    say(f"[parity] batch size limit {lim}")
    assert 8192 <= lim <= 16384
    g = gg.plant(gg.subtree(lim - 12, lim // 4, 8, 31), 12, 32)  # exactly the limit
    assert g.n == lim
    check_batch([g, gg.gnp(300, 0.02, 33)], tag="at the size limit")
    # one above: the 1024-lane tier takes it
    big = gg.from_edges(lim + 1, [(i, i + 1) for i in range(lim)] + [(0, lim)], "C_lim+1")
    check_batch([big, gg.gnp(200, 0.05, 34)], tag="one above the 256-lane tier")


def test_batch_large_tier_heavy_steps():
    """The 1,024-lane batch tier on n = 65,536 split graphs with heavy steps
    (class tables in L2), beside small graphs."""
    graphs = [heavy_split(32), moved_clique(21568), heavy_split(512), gg.gnp(700, 8 / 699, 31),
              gg.subtree(3000, 750, 8, 32)]
    check_batch(graphs, tag="1024-lane tier, heavy split graphs")


def test_batch_large_tier_with_plan_and_one_shot():
    graphs = [gg.plant(gg.subtree(20000, 5000, 12, 41), 9, 42),   # compact LDS state
              gg.gnp(17000, 0.0005, 43),
              gg.subtree(40000, 10000, 8, 44)]                      # class tables in global memory
    graphs += gg.config_batch(count=40, lo=32, hi=4096, seed=45)
    refs = [oracle.chordal_test(g) for g in graphs]
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    say("[parity] batch with the 1024-lane tier, one-shot")
    rs = lx.chordal_test_batch(dgs, outputs=True)
    say("[parity] batch with the 1024-lane tier, plan (side stream), two launches")
    plan = lx.BatchPlan(dgs, outputs=True)
    plan.launch()
    plan.launch()
    torch.cuda.synchronize()
    rp = plan.results()
    for g, ref, a, b in zip(graphs, refs, rs, rp):
        for r in (a, b):
            assert np.array_equal(r.order.cpu().numpy(), ref.order), g.name
            assert np.array_equal(r.parent.cpu().numpy(), ref.parent), g.name
            assert r.chordal == ref.chordal and r.witness == ref.witness, g.name
            assert r.cycle_list == ref.cycle.tolist(), g.name
    plan.close()


# ---------------------------------------------------------------------------
# Sizes around every team-size, chunk and layout boundary
# ---------------------------------------------------------------------------

BOUNDARY_SIZES = [63, 64, 65, 127, 129, 511, 512, 513, 1023, 1024, 1025, 2047, 2049, 4095, 4096, 4097, 8191,
                  8193, 16383, 16385, 32767, 32769]


def boundary_graphs(n, seed):
    """A chordal graph, the same kind with a planted chordless 9-cycle, and a
    sparse G(n, p), each with exactly n vertices."""
    return [gg.subtree(n, max(2, n // 4), 8, seed), gg.plant(gg.subtree(n - 9, max(2, n // 4), 8, seed + 1), 9, seed + 2),
            gg.gnp(n, min(1.0, 6.0 / (n - 1)), seed + 3)]


@pytest.mark.parametrize("n", BOUNDARY_SIZES)
def test_team_boundary_sizes(n):
    """Single graphs at n = 2^k - 1, 2^k, 2^k + 1 (and chunk edges): every
    team size the single-graph path picks, a partial last chunk and a last
    bitset word holding one vertex."""
    for g in boundary_graphs(n, 1000 + n):
        check_single(g, tag="boundary")


def test_batch_team_boundary_sizes():
    """One batch holding every boundary size up to 8,193 (wavefront and
    workgroup teams, rows of under and over 64 words side by side), under the
    default and two other wavefront thresholds."""
    graphs = []
    for n in BOUNDARY_SIZES:
        if n <= 8193:
            graphs += boundary_graphs(n, 5000 + n)
    for tuning in (None, {"wave_max_n": 256}, {"wave_max_n": -1}):
        check_batch(graphs, tuning=tuning, tag="boundary sizes")
