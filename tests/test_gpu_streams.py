"""GPU: calls made on a side stream with sync=True return the finished
results (the binding waits for that stream, not the current one), and
temporaries they allocate stay reserved until the side stream is done."""
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


def churn():
    """Allocations on the current stream right after a side-stream call:
    they must not land on memory the side stream still uses."""
    junk = [torch.full((1 << 20,), 7, dtype=torch.int32, device=DEV) for _ in range(8)]
    return sum(int(j[0]) for j in junk)


def test_side_stream_results():
    side = torch.cuda.Stream()
    graphs = [gg.intervals(6000, 10, 3), gg.intervals(6000, 10, 4, unit=False), gg.plant(gg.subtree(8000, 2000, 8, 5), 6, 6)]
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    torch.cuda.synchronize()
    for g, dg in zip(graphs, dgs):
        print(f"[streams] {g.name} n={g.n}", flush=True)
        r = lx.unit_interval_test(dg, stream=side)
        churn()
        ref = oracle.unit_interval_test(g)
        assert r.unit_interval == ref.unit_interval and r.witness == ref.witness
        side.synchronize()
        assert np.array_equal(r.order.cpu().numpy(), ref.order)
        c = lx.chordal_test(dg, stream=side)
        churn()
        ref = oracle.chordal_test(g)
        assert c.chordal == ref.chordal and c.witness == ref.witness
        side.synchronize()
        assert np.array_equal(c.order.cpu().numpy(), ref.order) and c.cycle_list == ref.cycle.tolist()
        order, rank, parent = lx.lexbfs_order(dg, stream=side)
        churn()
        side.synchronize()
        assert np.array_equal(order.cpu().numpy(), oracle.lexbfs(g).order)
    rs = lx.unit_interval_test_batch(dgs, stream=side, outputs=True)
    churn()
    for g, r in zip(graphs, rs):
        ref = oracle.unit_interval_test(g)
        assert r.unit_interval == ref.unit_interval and r.witness == ref.witness
    rs = lx.chordal_test_batch(dgs, stream=side, outputs=True)
    churn()
    side.synchronize()
    for g, r in zip(graphs, rs):
        ref = oracle.chordal_test(g)
        assert r.chordal == ref.chordal and r.witness == ref.witness
        assert np.array_equal(r.order.cpu().numpy(), ref.order)
