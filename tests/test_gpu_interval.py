"""GPU parity of multi-sweep LexBFS (LexBFS+, lexbfs_plus_order) and of the
three-sweep unit interval test (unit_interval_test) against the oracle,
element by element: every sweep's order, rank and parent, the verdict, the
third order and the witness triple."""
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


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check_plus(g, prev, tag=""):
    say(f"[plus] {tag} {g.name} n={g.n} m={g.m}")
    ref = oracle.lexbfs_plus(g, prev)
    d = lx.DeviceGraph.from_host(g, DEV)
    order, rank, parent = lx.lexbfs_plus(d, torch.from_numpy(np.ascontiguousarray(prev, dtype=np.int32)).to(DEV))
    assert np.array_equal(order.cpu().numpy(), ref.order), f"order {g.name}"
    assert np.array_equal(rank.cpu().numpy(), ref.rank), f"rank {g.name}"
    assert np.array_equal(parent.cpu().numpy(), ref.parent), f"parent {g.name}"


def check_interval(g, tag=""):
    say(f"[interval] {tag} {g.name} n={g.n} m={g.m}")
    ref = oracle.unit_interval_test(g)
    r = lx.unit_interval_test(lx.DeviceGraph.from_host(g, DEV))
    assert r.unit_interval == ref.unit_interval, f"verdict {g.name}"
    assert np.array_equal(r.order.cpu().numpy(), ref.order), f"third order {g.name}"
    assert r.witness == ref.witness, f"witness {g.name}: {r.witness} vs {ref.witness}"
    assert r.res_raw[4:].tolist() == [0, 0, 0, 0]
    return r


@pytest.mark.parametrize("idx", range(len(structured_cases())))
def test_structured(idx):
    g = structured_cases()[idx]
    rng = np.random.default_rng(idx)
    check_plus(g, rng.permutation(g.n).astype(np.int32), tag="structured")
    check_plus(g, np.arange(g.n, dtype=np.int32), tag="structured identity")
    check_interval(g, tag="structured")


@pytest.mark.parametrize("seed", range(3))
def test_random_plus(seed):
    rng = np.random.default_rng(100 + seed)
    for g in (gg.gnp(700, 0.02, 10 + seed), gg.gnp(4097, 0.003, 20 + seed), gg.subtree(3000, 700, 10, 30 + seed),
              gg.intervals(2000, 8, 40 + seed), gg.intervals(9000, 16, 50 + seed, unit=False)):
        check_plus(g, rng.permutation(g.n).astype(np.int32), tag="random prev")
        check_plus(g, oracle.lexbfs(g).order, tag="after LexBFS")


@pytest.mark.parametrize("seed", range(4))
def test_generated_intervals(seed):
    for n, deg in ((64, 6), (500, 10), (3000, 12), (12000, 20)):
        r = check_interval(gg.intervals(n, deg, 200 + seed), tag="unit")
        assert r.unit_interval
        check_interval(gg.intervals(n, deg, 300 + seed, unit=False), tag="mixed lengths")


@pytest.mark.parametrize("seed", range(2))
def test_other_families(seed):
    check_interval(gg.gnp(1500, 0.004, 70 + seed), tag="gnp")
    check_interval(gg.subtree(2000, 500, 8, 80 + seed), tag="subtree")
    for g in gg.split_pair(40, 400, 6, 90 + seed):
        check_interval(g, tag="split")


def test_full_size():
    """n = 65,536 (the largest supported size): the global-table LexBFS form
    in all three sweeps."""
    check_interval(gg.intervals(65536, 12, 3), tag="N=65536 unit")
    check_interval(gg.intervals(65536, 12, 4, unit=False), tag="N=65536 mixed")
    g = gg.gnp(65536, 0.0002, 5)
    check_plus(g, gg.permutation(g.n, 6), tag="N=65536 gnp")


def test_compact_layout_sizes():
    """n = 25,000 and 32,768: the compact LDS form of the LexBFS kernel (class
    ends from the class-start bitmap) in every sweep. n = 20,000 on 512 lanes
    is the largest LDS-table case (162,640 bytes of LDS, 64 vertices per
    lane) for the LexBFS+ sweep."""
    check_interval(gg.intervals(25000, 10, 31), tag="N=25000 unit")
    check_interval(gg.intervals(32768, 10, 32, unit=False), tag="N=32768 mixed")
    g = gg.gnp(20000, 0.0005, 33)
    check_plus(g, gg.permutation(g.n, 34), tag="N=20000 gnp")


def test_prev_not_a_permutation():
    """The device detects a prev_order that is not a permutation and fills
    the outputs with -1."""
    g = gg.gnp(300, 0.05, 9)
    d = lx.DeviceGraph.from_host(g, DEV)
    for prev in (np.zeros(g.n, dtype=np.int32), np.arange(g.n, dtype=np.int32) + 1):
        say(f"[plus] invalid prev {prev[:3].tolist()}")
        order, rank, parent = lx.lexbfs_plus(d, torch.from_numpy(prev).to(DEV))
        for t in (order, rank, parent):
            assert (t.cpu().numpy() == -1).all()
    check_plus(g, gg.permutation(g.n, 4), tag="valid prev after invalid ones")


def test_workspace_and_stream_reuse():
    """Back-to-back calls on one workspace on a side stream give the
    oracle's results each time."""
    graphs = [gg.intervals(1000, 8, 11), gg.intervals(5000, 10, 12, unit=False), gg.gnp(800, 0.01, 13)]
    lib = lx._lib.load()
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    need = max(int(lib.unit_interval_workspace_bytes(d.n, d.nnz)) for d in dgs)
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    rs = [lx.unit_interval_test(d, stream=s, ws=ws, sync=False) for d in dgs]
    s.synchronize()
    for g, r in zip(graphs, rs):
        ref = oracle.unit_interval_test(g)
        raw = r.res_raw.tolist()
        assert bool(raw[0]) == ref.unit_interval and tuple(raw[1:4]) == ref.witness, g.name
        assert np.array_equal(r.order.cpu().numpy(), ref.order), g.name


def check_batch(graphs, tag, outputs=True):
    say(f"[interval batch] {tag} count={len(graphs)} sum_n={sum(g.n for g in graphs)}")
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    rs = lx.unit_interval_test_batch(dgs, outputs=outputs)
    for g, r in zip(graphs, rs):
        ref = oracle.unit_interval_test(g)
        assert r.unit_interval == ref.unit_interval, f"verdict {g.name}"
        assert r.witness == ref.witness, f"witness {g.name}: {r.witness} vs {ref.witness}"
        if outputs:
            assert np.array_equal(r.order.cpu().numpy(), ref.order), f"third order {g.name}"
        assert r.res_raw[4:].tolist() == [0, 0, 0, 0]
    return rs


def test_batch_mix():
    """Mixed sizes and kinds, with empty, one-vertex and structured graphs:
    wavefront and workgroup teams in the same passes."""
    graphs = gg.config_interval_batch(count=150, lo=32, hi=4096, seed=3)
    graphs += [gg.from_edges(0, []), gg.from_edges(1, []), gg.from_edges(6, [(i, (i + 1) % 6) for i in range(6)])]
    graphs += structured_cases()[::5]
    check_batch(graphs, "mix")


def test_batch_large_tier():
    """Graphs above lexbfs_batch_max_n() run on the 1024-lane tier."""
    big = lx._lib.load().lexbfs_batch_max_n() + 500
    graphs = [gg.intervals(big, 10, 21), gg.intervals(big + 7, 10, 22, unit=False), gg.intervals(700, 8, 23)]
    check_batch(graphs, f"large tier n={big}")


def test_batch_equals_single():
    graphs = gg.config_interval_batch(count=40, lo=64, hi=2048, seed=5)
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    rs = lx.unit_interval_test_batch(dgs, outputs=True)
    for d, r in zip(dgs, rs):
        one = lx.unit_interval_test(d)
        assert one.unit_interval == r.unit_interval and one.witness == r.witness
        assert torch.equal(one.order, r.order)


def test_batch_full_workload():
    """The benchmark's 4,096-graph interval batch, every verdict and witness
    against the oracle; the third orders on an evenly spaced sample."""
    graphs = gg.config_interval_batch()
    rs = check_batch(graphs, "N log-uniform [32, 4096] x 4096", outputs=False)
    assert sum(r.unit_interval for r in rs) > 0
    sample = graphs[::64]
    check_batch(sample, "sample with orders")


BOUNDARY_SIZES = [63, 64, 65, 127, 129, 511, 512, 513, 1000, 1023, 1024, 1025, 2047, 2049, 4095, 4096, 4097,
                  8191, 8193]


@pytest.mark.parametrize("n", BOUNDARY_SIZES)
def test_interleaved_order_at_team_boundaries(n):
    """Sizes around every team-size and chunk boundary: the renamed sweeps
    deal ranks across lanes with a partial last chunk (cl < K) and n not a
    multiple of 64."""
    rng = np.random.default_rng(n)
    g = gg.gnp(n, min(1.0, 6.0 / max(n - 1, 1)), 500 + n)
    check_plus(g, rng.permutation(n).astype(np.int32), tag="boundary gnp")
    check_interval(gg.intervals(n, 6, 600 + n), tag="boundary unit")
    check_interval(gg.intervals(n, 6, 700 + n, unit=False), tag="boundary mixed")


def test_batch_at_team_boundaries():
    """A batch whose sizes straddle the wavefront / workgroup threshold and
    the chunk sizes of both team kinds."""
    graphs = []
    for n in BOUNDARY_SIZES:
        graphs.append(gg.intervals(n, 6, 800 + n))
        graphs.append(gg.intervals(n, 6, 900 + n, unit=False))
    check_batch(graphs, "boundary sizes")
