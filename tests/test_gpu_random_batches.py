"""Randomised batch parity: each batch mixes graph families (sparse and dense
G(n, p), subtree graphs with and without a planted chordless cycle, unit and
mixed-length interval graphs, paths followed by isolated vertices, empty
graphs), sizes log-uniform on [1, 12,000] and a random wavefront threshold;
every graph's LexBFS and MCS results and its unit interval verdict, witness
and third order are compared with the oracle. Seeded, so each run checks the
same batches; `RANDOM_BATCHES` sets how many."""
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
BATCHES = int(os.environ.get("RANDOM_BATCHES", "12"))


def rand_graph(rng, seed):
    n = int(np.exp(rng.uniform(0.0, np.log(12000))))
    kind = int(rng.integers(0, 7))
    if n < 3:
        return gg.from_edges(n, [], f"E{n}")
    if kind == 0:
        return gg.gnp(n, min(1.0, rng.uniform(0.3, 12) / (n - 1)), seed)
    if kind == 1:
        return gg.subtree(n, max(1, n // int(rng.integers(2, 8))), int(rng.integers(2, 12)), seed)
    if kind == 2 and n > 20:
        return gg.plant(gg.subtree(n - 9, max(1, (n - 9) // 4), 8, seed), 9, seed + 1)
    if kind == 3:
        return gg.intervals(n, rng.uniform(0.5, 20), seed, unit=bool(rng.integers(0, 2)))
    if kind == 4 and n <= 3000:
        return gg.gnp(n, rng.uniform(0.2, 0.9), seed)
    if kind == 5:
        return gg.from_edges(n, [(v, v + 1) for v in range(min(n - 1, int(rng.integers(1, n))))], f"P+E{n}")
    return gg.gnp(n, min(1.0, 2.0 / (n - 1)), seed)


@pytest.mark.parametrize("b", range(BATCHES))
def test_random_batch(b):
    rng = np.random.default_rng(1000 + b)
    count = int(rng.integers(1, 120))
    graphs = [rand_graph(rng, int(rng.integers(1, 1 << 30))) for _ in range(count)]
    tuning = [None, {"wave_max_n": -1}, {"wave_max_n": int(rng.integers(64, 1025))}][int(rng.integers(0, 3))]
    print(f"[random] batch {b} count={count} max_n={max(g.n for g in graphs)} tuning={tuning}", flush=True)
    sys.stdout.flush()
    dgs = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    for ordering, flags in (("lexbfs", 0), ("mcs", lx.LEXBFS_FLAG_MCS)):
        rs = lx.chordal_test_batch(dgs, outputs=True, flags=flags, tuning=tuning)
        for g, r in zip(graphs, rs):
            ref = oracle.chordal_test(g, ordering)
            assert np.array_equal(r.order.cpu().numpy(), ref.order), f"{ordering} order {g.name}"
            assert r.chordal == ref.chordal and r.witness == ref.witness, f"{ordering} verdict {g.name}"
            assert r.cycle_list == ref.cycle.tolist(), f"{ordering} certificate {g.name}"
    for g, r in zip(graphs, lx.unit_interval_test_batch(dgs, outputs=True)):
        ref = oracle.unit_interval_test(g)
        assert r.unit_interval == ref.unit_interval and r.witness == ref.witness, f"interval {g.name}"
        assert np.array_equal(r.order.cpu().numpy(), ref.order), f"interval order {g.name}"
