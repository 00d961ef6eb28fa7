"""GPU parity of the Maximum Cardinality Search path (LEXBFS_FLAG_MCS)
against the oracle's MCS, element by element, single graphs and batches."""
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
from test_gpu_parity import structured_cases  # noqa: E402

DEV = "cuda:0"
MCS = lx.LEXBFS_FLAG_MCS


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def same(r, ref, name):
    assert np.array_equal(r.order.cpu().numpy(), ref.order), f"order {name}"
    assert np.array_equal(r.rank.cpu().numpy(), ref.rank), f"rank {name}"
    assert np.array_equal(r.parent.cpu().numpy(), ref.parent), f"parent {name}"
    assert r.chordal == ref.chordal and r.witness == ref.witness, f"verdict/witness {name}"
    assert r.cycle_list == ref.cycle.tolist() and r.fallback == ref.fallback, f"certificate {name}"


def check(g, flags=0, tag=""):
    say(f"[mcs] {tag} {g.name} n={g.n} m={g.m}")
    ref = oracle.chordal_test(g, "mcs")
    r = lx.chordal_test(lx.DeviceGraph.from_host(g, DEV), flags=MCS | flags)
    same(r, ref, g.name)


@pytest.mark.parametrize("idx", range(len(structured_cases())))
def test_structured(idx):
    check(structured_cases()[idx], tag="structured")


@pytest.mark.parametrize("seed", range(3))
def test_random(seed):
    check(gg.gnp(900, 0.01, 60 + seed), tag="gnp")
    check(gg.gnp(5000, 0.002, 63 + seed), tag="gnp")
    check(gg.plant(gg.subtree(3000, 700, 10, seed), 5 + seed, seed), tag="planted")
    for g in gg.split_pair(60, 600, 8, 66 + seed):
        check(g, tag="split")


def test_large_sizes():
    for g in gg.config_single_large():
        check(g, tag="N=16384 workload")
    check(gg.plant(gg.subtree(30000, 8000, 10, 7), 7, 8), tag="n=30007")
    for g in gg.config_worst_steps():
        check(g, tag="N=65536 split workload")


def test_per_step_with_mcs_is_rejected():
    g = gg.gnp(50, 0.1, 1)
    with pytest.raises(lx.LexbfsError):
        lx.chordal_test(lx.DeviceGraph.from_host(g, DEV), flags=MCS | lx.LEXBFS_FLAG_PER_STEP)


def test_batch():
    graphs = gg.config_batch(count=80, lo=32, hi=4096, seed=12)
    graphs += [gg.from_edges(0, []), gg.from_edges(1, []), gg.from_edges(6, [(i, (i + 1) % 6) for i in range(6)]),
               gg.plant(gg.subtree(20000, 5000, 10, 13), 6, 14)]  # one on the 1024-lane tier
    say(f"[mcs] batch count={len(graphs)}")
    refs = [oracle.chordal_test(g, "mcs") for g in graphs]
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    for tuning in (None, {"wave_max_n": -1}):
        rs = lx.chordal_test_batch(dgs, outputs=True, flags=MCS, tuning=tuning)
        for g, r, ref in zip(graphs, rs, refs):
            same(r, ref, g.name)
    plan = lx.BatchPlan(dgs, outputs=True, flags=MCS)
    plan.launch()
    torch.cuda.synchronize()
    for g, r, ref in zip(graphs, plan.results(), refs):
        same(r, ref, g.name)
    plan.close()


def test_batch_forced_fallback():
    graphs = [gg.gnp(120, 0.05, 20 + s) for s in range(4)]
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    rs = lx.chordal_test_batch(dgs, outputs=True, flags=MCS | lx.LEXBFS_FLAG_FORCE_FALLBACK)
    for g, dg, r in zip(graphs, dgs, rs):
        s = lx.chordal_test(dg, flags=MCS | lx.LEXBFS_FLAG_FORCE_FALLBACK)
        assert r.witness == s.witness and r.cycle_list == s.cycle_list and r.fallback == s.fallback
        ref = oracle.chordal_test(g, "mcs")
        if not ref.chordal:
            cyc, fb = oracle.certificate(g, ref.order, ref.rank, ref.witness, force_fallback=True)
            assert r.cycle_list == cyc.tolist() and fb


@pytest.mark.parametrize("n", [63, 65, 511, 513, 1023, 1025, 2049, 4095, 4097, 8193, 16385, 32769])
def test_team_boundary_sizes(n):
    """MCS on single graphs at team-size and chunk boundaries."""
    check(gg.subtree(n, max(2, n // 4), 8, 6000 + n), tag="boundary")
    check(gg.plant(gg.subtree(n - 9, max(2, n // 4), 8, 6001 + n), 9, 6002 + n), tag="boundary planted")
    check(gg.gnp(n, 6.0 / (n - 1), 6003 + n), tag="boundary gnp")


def test_batch_team_boundary_sizes():
    graphs = []
    for n in (63, 65, 511, 513, 1023, 1025, 2047, 2049, 4095, 4097, 8191, 8193):
        graphs += [gg.subtree(n, max(2, n // 4), 8, 7000 + n), gg.plant(gg.subtree(n - 9, max(2, n // 4), 8, 7001 + n), 9, 7002 + n),
                   gg.gnp(n, 6.0 / (n - 1), 7003 + n)]
    say(f"[mcs] boundary batch count={len(graphs)}")
    refs = [oracle.chordal_test(g, "mcs") for g in graphs]
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    for tuning in (None, {"wave_max_n": -1}):
        rs = lx.chordal_test_batch(dgs, outputs=True, flags=MCS, tuning=tuning)
        for g, r, ref in zip(graphs, rs, refs):
            same(r, ref, g.name)
