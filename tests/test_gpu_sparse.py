"""GPU parity on very sparse graphs (average degree 0.5-2, components
followed by isolated vertices). When a pivot empties the top class, the
class below is often a large class of untouched vertices whose start lies
more than two bitmap words below the top position, so the step falls back to
the team-wide scan of the class-start bitmap (a second reduction). Denser
graphs almost never reach that path. Chordality (LexBFS, MCS and the
per-step-launch form), LexBFS+ and the unit interval test, single graphs in
every LexBFS layout and batches on wavefront and workgroup teams, against
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
from test_gpu_interval import check_batch as check_interval_batch  # noqa: E402
from test_gpu_interval import check_interval, check_plus  # noqa: E402
from test_gpu_mcs import check as check_mcs  # noqa: E402
from test_gpu_parity import check_batch, check_single  # noqa: E402

DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def path_then_isolated(n, L):
    return gg.from_edges(n, [(v, v + 1) for v in range(L - 1)], f"P{L}+E{n - L}")


def clique_then_isolated(n, k):
    return gg.from_edges(n, [(u, v) for u in range(k) for v in range(u + 1, k)], f"K{k}+E{n - k}")


def sparse_gnp(n, deg, seed):
    return gg.gnp(n, deg / (n - 1), seed)


# n = 700 and 3,000: LDS tables (128- and 256-lane teams); 9,000: 512 lanes;
# 25,000: compact LDS layout; 40,000: class tables in L2.
SINGLE = [(700, 1.0, 1), (1000, 0.5, 2), (3000, 1.5, 3), (9000, 2.0, 4), (25000, 1.0, 5), (40000, 1.5, 6)]


@pytest.mark.parametrize("n,deg,seed", SINGLE)
def test_sparse_single(n, deg, seed):
    g = sparse_gnp(n, deg, seed)
    check_single(g, tag="sparse")
    if n <= 9000:
        check_single(g, flags=lx.LEXBFS_FLAG_PER_STEP, tag="sparse, per-step launches")
    check_mcs(g, tag="sparse")


@pytest.mark.parametrize("case", ["path", "clique", "star"])
def test_components_then_isolated(case):
    g = {"path": lambda: path_then_isolated(1500, 100), "clique": lambda: clique_then_isolated(2050, 50),
         "star": lambda: gg.from_edges(801, [(0, v) for v in range(1, 301)], "S300+E500")}[case]()
    check_single(g, tag="components")
    check_single(g, flags=lx.LEXBFS_FLAG_PER_STEP, tag="components, per-step launches")
    check_mcs(g, tag="components")
    check_interval(g, tag="components")


def test_sparse_batch():
    """Sparse graphs of every size class in one batch, under the default
    wavefront threshold, workgroups only and a low threshold; LexBFS and MCS."""
    graphs = [sparse_gnp(n, d, 100 + n) for n in (40, 200, 500, 900, 1024, 1500, 2500, 4000) for d in (0.5, 1.5)]
    graphs += [path_then_isolated(1500, 100), clique_then_isolated(2050, 50), path_then_isolated(600, 70)]
    for tuning in (None, {"wave_max_n": -1}, {"wave_max_n": 256}):
        check_batch(graphs, tuning=tuning, tag="sparse")
    refs = [oracle.chordal_test(g, "mcs") for g in graphs]
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    say("[sparse] MCS batch")
    rs = lx.chordal_test_batch(dgs, outputs=True, flags=lx.LEXBFS_FLAG_MCS)
    for g, r, ref in zip(graphs, rs, refs):
        assert np.array_equal(r.order.cpu().numpy(), ref.order), g.name
        assert r.chordal == ref.chordal and r.witness == ref.witness, g.name


@pytest.mark.parametrize("n,deg,seed", [(700, 1.0, 7), (3000, 1.5, 8), (9000, 2.0, 9)])
def test_sparse_multi_sweep(n, deg, seed):
    g = sparse_gnp(n, deg, seed)
    check_plus(g, gg.permutation(n, seed + 1), tag="sparse")
    check_interval(g, tag="sparse")


def test_sparse_interval_batch():
    graphs = [sparse_gnp(n, 1.0, 200 + n) for n in (100, 700, 1500, 3000)]
    graphs += [path_then_isolated(1500, 100), gg.intervals(2000, 1.0, 17), gg.intervals(900, 0.5, 18, unit=False)]
    check_interval_batch(graphs, "sparse")


def test_batch_with_a_maximum_size_graph():
    """A batch holding an n = 65,536 graph (the largest supported size: the
    1,024-lane tier with its class tables in L2) beside small ones, for
    LexBFS, MCS and the batched unit interval test."""
    big = sparse_gnp(65536, 1.5, 300)
    graphs = [big, sparse_gnp(900, 1.0, 301), sparse_gnp(3000, 1.5, 302), path_then_isolated(1500, 100)]
    check_batch(graphs, tag="with n = 65536")
    refs = [oracle.chordal_test(g, "mcs") for g in graphs]
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    say("[sparse] MCS batch with n = 65536")
    rs = lx.chordal_test_batch(dgs, outputs=True, flags=lx.LEXBFS_FLAG_MCS)
    for g, r, ref in zip(graphs, rs, refs):
        assert np.array_equal(r.order.cpu().numpy(), ref.order), g.name
        assert r.chordal == ref.chordal and r.witness == ref.witness, g.name
    check_interval_batch(graphs, "with n = 65536")
