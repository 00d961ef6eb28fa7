"""Serving on the GPU: every request's result equals the oracle's and the
single-graph call's, whatever else shares its batch."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1508_06329_amd as lx  # noqa: E402
from paper_1508_06329_amd import serving  # noqa: E402


def stream(count, lo, hi, seed):
    ns, kinds, Ls, gaps = gg.mix_specs(count, lo, hi, seed)
    graphs = [gg.mix_graph(int(ns[i]), int(kinds[i]), int(Ls[i]), gg.graph_seed(seed, 1000 + i)) for i in range(count)]
    return graphs, np.cumsum(gaps)


def check(out, graphs):
    assert out["completed"] == len(graphs) and out["rejected"] == 0
    for r in out["requests"]:
        if r.result is None:
            continue
        ref = oracle.chordal_test(graphs[r.rid])
        assert r.result.chordal == ref.chordal and r.result.witness == ref.witness, r.rid
        assert r.result.cycle_list == ref.cycle.tolist(), r.rid
        assert np.array_equal(r.result.order.cpu().numpy(), ref.order), r.rid


@pytest.mark.parametrize("tight", [True, False])
def test_serving_matches_oracle(tight):
    graphs, arr = stream(48, 64, 3000, 3)
    graphs.append(gg.plant(gg.subtree(16500, 4000, 8, 9), 6, 10))  # above the batch limit
    arr = np.append(arr * 1e-3, 0.01)
    big = max(serving.footprint_bytes(g.n, g.nnz, g.W) for g in graphs)
    budget = int(1.1 * big) if tight else 1 << 30  # tight: requests queue behind the largest
    print(f"[serving] budget={budget} requests={len(graphs)}", flush=True)
    out = serving.serve(graphs, arr, budget_bytes=budget, outputs=True)
    check(out, graphs)
    assert out["peak_bytes"] <= budget


def test_serving_rejects_oversize():
    graphs, arr = stream(6, 64, 500, 7)
    graphs.append(gg.subtree(5000, 1000, 8, 8))
    small = max(serving.footprint_bytes(g.n, g.nnz, g.W) for g in graphs[:-1])
    out = serving.serve(graphs, np.zeros(len(graphs)), budget_bytes=small, outputs=True)
    assert out["rejected"] == 1 and out["completed"] == 6


def test_serial_path_matches_oracle():
    graphs, arr = stream(16, 64, 2000, 4)
    print(f"[serving] serial requests={len(graphs)}", flush=True)
    out = serving.serve(graphs, arr * 1e-3, serial=True, outputs=True)
    check(out, graphs)


def test_same_result_alone_and_in_mix():
    graphs, arr = stream(24, 64, 2000, 5)
    out = serving.serve(graphs, np.zeros(len(graphs)), outputs=True)  # all at once: one big mix
    for r in out["requests"]:
        alone = lx.chordal_test(lx.DeviceGraph.from_host(graphs[r.rid]))
        assert alone.chordal == r.result.chordal and alone.witness == r.result.witness
        assert alone.cycle_list == r.result.cycle_list
        assert torch.equal(alone.order, r.result.order)


@pytest.mark.parametrize("seed", range(3))
def test_random_streams(seed):
    """Requests drawn as in the random batch test (mixed families and
    densities, sizes up to 12,000, some above the batch limit), random gaps
    between arrivals, and a tight or a loose memory budget."""
    from test_gpu_random_batches import rand_graph

    rng = np.random.default_rng(7000 + seed)
    count = int(rng.integers(10, 60))
    graphs = [g for g in (rand_graph(rng, int(rng.integers(1, 1 << 30))) for _ in range(count)) if g.n > 0]
    arr = np.cumsum(rng.exponential(rng.uniform(1e-5, 2e-3), len(graphs)))
    big = max(serving.footprint_bytes(g.n, g.nnz, g.W) for g in graphs)
    budget = int(big * rng.uniform(1.0, 1.5)) if rng.random() < 0.5 else 1 << 30
    print(f"[serving] random stream {seed}: {len(graphs)} requests, budget {budget}", flush=True)
    out = serving.serve(graphs, arr, budget_bytes=budget, outputs=True)
    check(out, graphs)
    assert out["peak_bytes"] <= budget


def test_serving_stream_spans_the_serving_sizes():
    """One stream whose sizes span the serving workload's whole range,
    N log-uniform on [64, 32768] with both ends present, every response
    checked against the oracle (order included)."""
    graphs, arr = stream(40, 64, 32768, 11)
    graphs.append(gg.mix_graph(64, 0, 0, gg.graph_seed(11, 5000)))
    graphs.append(gg.mix_graph(32768, 2, 9, gg.graph_seed(11, 5001)))
    graphs.append(gg.mix_graph(32768, 1, 0, gg.graph_seed(11, 5002)))
    arr = np.append(arr * 2e-3, [arr[-1] * 2e-3 + 0.001 * k for k in range(1, 4)])
    ns = sorted(g.n for g in graphs)
    print(f"[serving] full-range stream: {len(graphs)} requests, N from {ns[0]} to {ns[-1]}", flush=True)
    assert ns[0] == 64 and ns[-1] == 32768
    out = serving.serve(graphs, arr, budget_bytes=64 << 30, outputs=True)
    check(out, graphs)
