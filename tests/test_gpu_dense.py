"""GPU parity on dense graphs (half or all of the possible edges): neighbour
counts near n per class and per step, pivots that split every class, and
rows with every word full. The sparse workloads never reach these counts.
Chordality (LexBFS, MCS and the per-step-launch form), LexBFS+ and the
unit interval test, single graphs and batches, all element by element
against the oracle."""
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


def complete(n):
    return gg.gnp(n, 1.0, 1)


def dense_cases():
    """Chordal: K_n, K_n less one edge, a split graph (a 1,500-clique and
    1,500 independent vertices, each joined to 1,400 random clique vertices).
    Not chordal: G(n, 1/2), K_n less
    a perfect matching (every two removed edges leave an induced 4-cycle)."""
    kn = complete(3000)
    k1 = complete(1000)
    bits = k1.bits.reshape(1000, k1.W).copy()
    v = np.arange(1000)
    bits[v, (v ^ 1) >> 6] &= ~(np.uint64(1) << ((v ^ 1) & 63).astype(np.uint64))  # drop edges {2i, 2i + 1}
    km = gg.finish(1000, bits.reshape(-1), k1.W, "K1000 less a perfect matching")
    return [kn, gg.remove_edge(kn, 5, 2990), gg.split(1500, 1500, 1400, 3), gg.gnp(3000, 0.5, 4),
            gg.gnp(900, 0.5, 5), km]


@pytest.mark.parametrize("idx", range(6))
def test_dense_chordality(idx):
    g = dense_cases()[idx]
    check_single(g, tag="dense")
    check_single(g, flags=lx.LEXBFS_FLAG_PER_STEP, tag="dense, per-step launches")
    check_mcs(g, tag="dense")


def test_dense_batch():
    """Dense graphs on wavefront (n <= 1024) and workgroup teams, mixed with
    sparse ones, under the default threshold and workgroups only."""
    graphs = dense_cases() + [complete(700), gg.gnp(1024, 0.9, 6), gg.gnp(4096, 0.3, 7)]
    graphs += gg.config_batch(count=30, lo=32, hi=4096, seed=8)
    for tuning in (None, {"wave_max_n": -1}):
        check_batch(graphs, tuning=tuning, tag="dense")
    refs = [oracle.chordal_test(g, "mcs") for g in graphs]
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    say("[dense] MCS batch")
    rs = lx.chordal_test_batch(dgs, outputs=True, flags=lx.LEXBFS_FLAG_MCS)
    for g, r, ref in zip(graphs, rs, refs):
        assert np.array_equal(r.order.cpu().numpy(), ref.order), g.name
        assert r.chordal == ref.chordal and r.witness == ref.witness, g.name
        assert r.cycle_list == ref.cycle.tolist(), g.name


@pytest.mark.parametrize("case", ["K2000", "gnp2000_half", "unit_long", "mixed_long"])
def test_dense_multi_sweep(case):
    g = {"K2000": lambda: complete(2000), "gnp2000_half": lambda: gg.gnp(2000, 0.5, 9),
         "unit_long": lambda: gg.intervals(2500, 800, 10), "mixed_long": lambda: gg.intervals(2500, 800, 11, unit=False)}[case]()
    check_plus(g, gg.permutation(g.n, 12), tag="dense")
    check_interval(g, tag="dense")


def test_dense_interval_batch():
    graphs = [complete(1500), gg.gnp(900, 0.5, 13), gg.intervals(2000, 600, 14), gg.intervals(1000, 500, 15, unit=False),
              gg.intervals(3000, 8, 16)]
    check_interval_batch(graphs, "dense")
