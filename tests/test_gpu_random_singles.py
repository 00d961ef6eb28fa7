"""Randomised single-graph parity: graphs drawn as in the random batch test,
plus (about one in seven) sparse G(n, p) or interval graphs of 12,000-65,536
vertices, so that every single-graph LexBFS layout runs (LDS tables, compact,
class tables in L2). Each graph: LexBFS and MCS results (order, parents,
verdict, witness, certificate), the per-step-launch form up to n = 9,000,
LexBFS+ after a random previous order, the unit interval test, and the
bitset built on the device from the CSR (with padded rows) and the whole
path from that CSR, against the oracle. Seeded; `RANDOM_SINGLES` sets how
many."""
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
from test_gpu_random_batches import rand_graph  # noqa: E402

DEV = "cuda:0"
COUNT = int(os.environ.get("RANDOM_SINGLES", "40"))


@pytest.mark.parametrize("k", range(COUNT))
def test_random_single(k):
    rng = np.random.default_rng(5000 + k)
    if rng.random() < 0.15:
        n = int(rng.integers(12000, 65537))
        seed = int(rng.integers(1, 1 << 30))
        g = (gg.gnp(n, rng.uniform(0.5, 6) / (n - 1), seed) if rng.random() < 0.5
             else gg.intervals(n, rng.uniform(1, 12), seed, unit=bool(rng.integers(0, 2))))
    else:
        g = rand_graph(rng, int(rng.integers(1, 1 << 30)))
    print(f"[random single] {k} {g.name} n={g.n} m={g.m}", flush=True)
    sys.stdout.flush()
    d = lx.DeviceGraph.from_host(g, DEV)
    for ordering, flags in (("lexbfs", 0), ("mcs", lx.LEXBFS_FLAG_MCS)):
        r = lx.chordal_test(d, flags=flags)
        ref = oracle.chordal_test(g, ordering)
        assert np.array_equal(r.order.cpu().numpy(), ref.order), f"{ordering} order"
        assert np.array_equal(r.parent.cpu().numpy(), ref.parent), f"{ordering} parent"
        assert r.chordal == ref.chordal and r.witness == ref.witness, f"{ordering} verdict"
        assert r.cycle_list == ref.cycle.tolist(), f"{ordering} certificate"
    if g.n <= 9000:
        r = lx.chordal_test(d, flags=lx.LEXBFS_FLAG_PER_STEP)
        ref = oracle.chordal_test(g)
        assert np.array_equal(r.order.cpu().numpy(), ref.order) and r.witness == ref.witness, "per-step"
    prev = rng.permutation(g.n).astype(np.int32)
    order, rank, parent = lx.lexbfs_plus(d, torch.from_numpy(prev).to(DEV))
    ref = oracle.lexbfs_plus(g, prev)
    assert np.array_equal(order.cpu().numpy(), ref.order) and np.array_equal(rank.cpu().numpy(), ref.rank), "LexBFS+"
    assert np.array_equal(parent.cpu().numpy(), ref.parent), "LexBFS+ parent"
    r = lx.unit_interval_test(d)
    ref = oracle.unit_interval_test(g)
    assert r.unit_interval == ref.unit_interval and r.witness == ref.witness, "unit interval"
    assert np.array_equal(r.order.cpu().numpy(), ref.order), "unit interval order"
    # Device-side ingestion: the bitset built from the CSR on the device (rows
    # padded by a random number of words) and the whole path from that CSR.
    if g.n > 0:
        pad = int(rng.integers(0, 4))
        W = (g.n + 63) // 64 + pad
        rp = torch.from_numpy(g.row_ptr).to(DEV)
        ci = torch.from_numpy(g.col_idx if g.col_idx.size else np.zeros(0, np.int32)).to(DEV)
        bits = lx.build_bitset(g.n, rp, ci, W)
        torch.cuda.synchronize()
        got = bits.cpu().numpy().view(np.uint64)[: g.n * W].reshape(g.n, W)
        assert np.array_equal(got, oracle.bitset_from_csr(g.n, g.row_ptr, g.col_idx, W)), "device bitset"
        r = lx.chordal_test(lx.DeviceGraph.from_csr(g.n, rp, ci))
        ref = oracle.chordal_test(g)
        assert np.array_equal(r.order.cpu().numpy(), ref.order) and r.witness == ref.witness, "from device CSR"
