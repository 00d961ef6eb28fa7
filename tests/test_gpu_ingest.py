"""GPU parity of the device-side bitset builder (lexbfs_build_bitset)
against the oracle's bitset definition, bit-exact, and the whole path from
a device CSR."""
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


def build(g, W):
    print(f"[ingest] {g.name} n={g.n} W={W}", flush=True)
    rp = torch.from_numpy(g.row_ptr).to(DEV)
    ci = torch.from_numpy(g.col_idx if g.col_idx.size else np.zeros(0, np.int32)).to(DEV)
    bits = lx.build_bitset(g.n, rp, ci, W)
    torch.cuda.synchronize()
    return bits.cpu().numpy().view(np.uint64)[: g.n * W].reshape(g.n, W), rp, ci


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 129, 1000, 4097])
@pytest.mark.parametrize("pad", [0, 3])
def test_builder_matches_definition(n, pad):
    g = gg.gnp(n, min(1.0, 12.0 / max(n - 1, 1)), n + pad) if n > 1 else gg.from_edges(1, [])
    W = (n + 63) // 64 + pad
    got, _, _ = build(g, W)
    assert np.array_equal(got, oracle.bitset_from_csr(g.n, g.row_ptr, g.col_idx, W))


def test_builder_structured_and_empty_rows():
    for g in (gg.from_edges(200, [(0, 199), (63, 64), (64, 127), (128, 191)]), gg.from_edges(300, []),
              gg.from_edges(90, [(a, b) for a in range(90) for b in range(a + 1, 90)]), gg.subtree(3000, 700, 10, 5)):
        got, _, _ = build(g, g.W)
        assert np.array_equal(got, oracle.bitset_from_csr(g.n, g.row_ptr, g.col_idx, g.W)), g.name


def test_builder_full_split_workload():
    g = gg.config_worst_steps()[1]
    got, _, _ = build(g, g.W)
    assert np.array_equal(got, oracle.bitset_from_csr(g.n, g.row_ptr, g.col_idx, g.W))


def test_whole_path_from_device_csr():
    for g in (gg.plant(gg.subtree(5000, 1200, 10, 9), 7, 9), gg.gnp(2000, 0.004, 10)):
        rp = torch.from_numpy(g.row_ptr).to(DEV)
        ci = torch.from_numpy(g.col_idx).to(DEV)
        dg = lx.DeviceGraph.from_csr(g.n, rp, ci)
        r = lx.chordal_test(dg)
        ref = oracle.chordal_test(g)
        assert np.array_equal(r.order.cpu().numpy(), ref.order)
        assert r.chordal == ref.chordal and r.witness == ref.witness and r.cycle_list == ref.cycle.tolist()


def test_whole_path_from_host_csr_on_a_side_stream():
    """Pinned staging and asynchronous CSR copies on a side stream, the
    bitset built there, and the test queued behind it on the same stream:
    bit-exact bitsets and the oracle's results, for graphs with and without
    edges."""
    side = torch.cuda.Stream()
    graphs = [gg.plant(gg.subtree(5000, 1200, 10, 11), 6, 11), gg.gnp(3000, 0.003, 12), gg.from_edges(70, [])]
    for g in graphs:
        print(f"[ingest] host CSR {g.name} n={g.n}", flush=True)
        dg = lx.DeviceGraph.from_host_csr(g, DEV, stream=side)
        r = lx.chordal_test(dg, stream=side)  # sync=True: waits on the side stream
        side.synchronize()
        bits = dg.bits.cpu().numpy().view(np.uint64)[: g.n * dg.W].reshape(g.n, dg.W)
        assert np.array_equal(bits, oracle.bitset_from_csr(g.n, g.row_ptr, g.col_idx, dg.W)), g.name
        ref = oracle.chordal_test(g)
        assert np.array_equal(r.order.cpu().numpy(), ref.order), g.name
        assert r.chordal == ref.chordal and r.witness == ref.witness and r.cycle_list == ref.cycle.tolist()
