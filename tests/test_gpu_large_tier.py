"""GPU: the batch tier for graphs above one 256-lane workgroup's LDS. Each
such graph runs on its own workgroup with the single-graph state: 512 lanes
up to 32,768 vertices (class tables in LDS while they fit, else the compact
layout), 1,024 lanes above (compact layout, else class tables in L2). A
batch holding graphs of every one of these forms beside small ones, for
LexBFS and MCS, through chordal_test_batch (one stream) and a prepared plan
(the two team sizes on streams of their own), element by element against
the oracle."""
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


def graphs_across_forms():
    tier = lx._lib.load().lexbfs_batch_max_n()
    gs = [gg.gnp(tier + 1, 8 / tier, 1),                               # 512 lanes, just above the 256-lane tier
          gg.plant(gg.subtree(18000, 4500, 8, 2), 7, 3),               # 512 lanes, class tables in LDS
          gg.gnp(26000, 6 / 25999, 4),                                 # 512 lanes, compact layout
          gg.subtree(32768, 8192, 8, 5),                               # 512 lanes at its largest n
          gg.gnp(32769, 8 / 32768, 6),                                 # 1,024 lanes at its smallest n
          gg.plant(gg.subtree(45000, 11250, 8, 7), 9, 8),              # 1,024 lanes, compact layout
          gg.gnp(65536, 3 / 65535, 9)]                                 # 1,024 lanes, class tables in L2
    gs += [gg.gnp(700, 8 / 699, 10), gg.subtree(3000, 750, 8, 11), gg.from_edges(1, []),
           gg.plant(gg.subtree(9000, 2250, 8, 12), 5, 13)]
    return gs


def check(graphs, rs, refs, tag):
    for g, r, ref in zip(graphs, rs, refs):
        assert np.array_equal(r.order.cpu().numpy(), ref.order), (tag, g.name)
        assert np.array_equal(r.rank.cpu().numpy(), ref.rank), (tag, g.name)
        assert np.array_equal(r.parent.cpu().numpy(), ref.parent), (tag, g.name)
        assert r.chordal == ref.chordal and r.witness == ref.witness, (tag, g.name)
        assert r.cycle_list == ref.cycle.tolist() and r.fallback == ref.fallback, (tag, g.name)


@pytest.mark.parametrize("ordering", ["lexbfs", "mcs"])
def test_large_tier_every_form(ordering):
    graphs = graphs_across_forms()
    flags = lx.LEXBFS_FLAG_MCS if ordering == "mcs" else 0
    refs = [oracle.chordal_test(g, ordering) for g in graphs]
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    say(f"[large tier] {ordering}: chordal_test_batch, n = {[g.n for g in graphs]}")
    check(graphs, lx.chordal_test_batch(dgs, outputs=True, flags=flags), refs, "one stream")
    say(f"[large tier] {ordering}: prepared plan, two launches")
    plan = lx.BatchPlan(dgs, outputs=True, flags=flags)
    for _ in range(2):
        plan.launch()
        torch.cuda.synchronize()
        check(graphs, plan.results(), refs, "plan")
    plan.close()


def test_large_tier_one_size_only():
    """Only 512-lane graphs, and only 1,024-lane graphs, each with and
    without small graphs beside them."""
    small = [gg.gnp(500, 8 / 499, 20)]
    mid = [gg.gnp(20000, 8 / 19999, 21), gg.plant(gg.subtree(30000, 7500, 8, 22), 6, 23)]
    big = [gg.gnp(40000, 4 / 39999, 24)]
    for graphs in (mid, mid + small, big, big + small):
        refs = [oracle.chordal_test(g) for g in graphs]
        dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
        say(f"[large tier] n = {[g.n for g in graphs]}")
        plan = lx.BatchPlan(dgs, outputs=True)
        plan.launch()
        torch.cuda.synchronize()
        check(graphs, plan.results(), refs, "plan")
        plan.close()
