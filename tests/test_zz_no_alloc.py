"""GPU: chordal_test_noalloc, whose scratch is the library's fixed device
array, gives exactly chordal_test's results (order, rank, parent, verdict,
witness, certificate, fallback flag) on calls in a row, each graph smaller
than the one before, so that every call starts from the previous call's
contents of the array."""
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1508_06329_amd as lx  # noqa: E402

DEV = "cuda:0"
KEYS = ("order", "rank", "parent", "cycle")


def via_noalloc(dg, flags):
    n = dg.n
    res = torch.full((8,), -7, dtype=torch.int32, device=DEV)
    outs = {k: torch.full((max(n, 1),), -7, dtype=torch.int32, device=DEV) for k in KEYS}
    lx.chordal_test_noalloc(dg, res, outs, flags=flags)
    torch.cuda.synchronize()
    return lx.Result.from_record(res, **{k: v[:n] for k, v in outs.items()})


def assert_same(got, ref):
    assert (got.chordal, got.witness, got.cycle_len, got.fallback) == (ref.chordal, ref.witness, ref.cycle_len,
                                                                      ref.fallback)
    for k in ("order", "rank", "parent"):
        assert torch.equal(getattr(got, k), getattr(ref, k)), k
    assert got.cycle_list == ref.cycle_list


def run_sequence(calls):
    for g, flags in calls:
        print(f"[noalloc] {g.name} n={g.n} flags={flags}", flush=True)
        dg = lx.DeviceGraph.from_host(g, DEV)
        ref = lx.chordal_test(dg, flags=flags)
        assert_same(via_noalloc(dg, flags), ref)


def test_two_calls_second_smaller():
    big, small = gg.config_single_large()[1], gg.config_single_small()[1]  # G(16384, 0.003); 1,029 with a C5
    run_sequence([(big, 0), (small, 0)])


def test_largest_graph_then_smaller_ones():
    # n = 65,536 (the scratch array's full size: class tables in the array),
    # then ever smaller graphs with MCS, the per-step form and the forced
    # fallback certificate, and an empty graph.
    split = gg.config_worst_steps()[1]
    calls = [(split, 0), (gg.plant(gg.subtree(9000, 2250, 8, 3), 9, 4), lx.LEXBFS_FLAG_MCS),
             (gg.config_single_small()[0], 0), (gg.plant(gg.subtree(700, 175, 8, 5), 6, 6), lx.LEXBFS_FLAG_PER_STEP),
             (gg.plant(gg.subtree(300, 75, 8, 7), 5, 8), lx.LEXBFS_FLAG_FORCE_FALLBACK), (gg.from_edges(1, []), 0),
             (gg.from_edges(0, []), 0)]
    run_sequence(calls)
