"""GPU: the input contract check (lexbfs_validate, LEXBFS_FLAG_VALIDATE).

Valid graphs of every family pass, and the validating calls give the same
results as the plain ones. Malformed graphs -- each broken in one way, with
every array still of the size the contract gives it, so that the check's
own reads stay in bounds -- come back as LEXBFS_EGRAPH naming the broken
rule, from lexbfs_validate, from chordal_test with the flag and from a
batch with the flag (naming the graph). A malformed graph is only ever
passed to the validating calls."""
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
EGRAPH = -4


def upload(n, W, rp, ci, bits):
    t_rp = torch.from_numpy(np.ascontiguousarray(rp, dtype=np.int32)).to(DEV)
    t_ci = torch.from_numpy(np.ascontiguousarray(ci, dtype=np.int32)).to(DEV)
    t_b = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint64).view(np.int64)).to(DEV)
    return lx.DeviceGraph(n, W, t_rp, t_ci, t_b)


def setbit(bits, W, v, u, on=True):
    w = v * W + (u >> 6)
    m = np.uint64(1) << np.uint64(u & 63)
    bits[w] = (bits[w] | m) if on else (bits[w] & ~m)


def base():
    g = gg.gnp(200, 0.05, 7)
    return g.n, g.W, g.row_ptr.copy(), g.col_idx.copy(), g.bits.copy()


def row_with(rp, k):
    """A vertex with at least k neighbours."""
    return int(np.nonzero(np.diff(rp) >= k)[0][0])


def break_graph(kind):
    n, W, rp, ci, bits = base()
    if kind == "asymmetric":          # (v, u) dropped from row v only
        v = row_with(rp, 2)
        u = int(ci[rp[v]])
        ci = np.delete(ci, rp[v])
        rp[v + 1:] -= 1
        setbit(bits, W, v, u, False)
        return n, W, rp, ci, bits, "not symmetric"
    if kind == "unsorted":
        v = row_with(rp, 2)
        ci[rp[v]], ci[rp[v] + 1] = ci[rp[v] + 1], ci[rp[v]]
        return n, W, rp, ci, bits, "not strictly ascending"
    if kind == "duplicate":
        v = row_with(rp, 3)
        ci[rp[v] + 1] = ci[rp[v]]
        return n, W, rp, ci, bits, "not strictly ascending"
    if kind == "self-loop":           # v added to its own row, CSR and bitset alike
        v = row_with(rp, 1)
        row = np.sort(np.append(ci[rp[v]:rp[v + 1]], v))
        ci = np.concatenate([ci[:rp[v]], row, ci[rp[v + 1]:]])
        rp[v + 1:] += 1
        setbit(bits, W, v, v)
        return n, W, rp, ci, bits, "self-loop"
    if kind == "extra-bit":           # an edge in the bitset only (both directions)
        v = row_with(rp, 1)
        u = next(u for u in range(n) if u != v and u not in set(ci[rp[v]:rp[v + 1]].tolist()))
        setbit(bits, W, v, u)
        setbit(bits, W, u, v)
        return n, W, rp, ci, bits, "bitset holds entries"
    if kind == "missing-bit":         # an edge in the CSR only (both directions)
        v = row_with(rp, 1)
        u = int(ci[rp[v]])
        setbit(bits, W, v, u, False)
        setbit(bits, W, u, v, False)
        return n, W, rp, ci, bits, "missing from the bitset"
    if kind == "id-n":                # the last entry of the last non-empty row becomes n
        v = int(np.nonzero(np.diff(rp) > 0)[0][-1])
        ci[rp[v + 1] - 1] = n
        return n, W, rp, ci, bits, "outside 0..n-1"
    if kind == "id-negative":
        v = row_with(rp, 1)
        ci[rp[v]] = -1
        return n, W, rp, ci, bits, "outside 0..n-1"
    if kind == "bit-beyond-n":        # n = 200: bit 200 of the last word set
        setbit(bits, W, 3, n)
        return n, W, rp, ci, bits, "bitset holds entries"
    if kind == "rowptr-start":
        rp[0] = 1
        return n, W, rp, ci, bits, "row pointers"
    if kind == "rowptr-end":          # one more col_idx entry than row_ptr[n] says
        ci = np.append(ci, 0)
        return n, W, rp, ci, bits, "row pointers"
    if kind == "rowptr-decreasing":
        v = row_with(rp, 1)
        rp[v + 1] = rp[v] - 1 if rp[v] > 0 else rp[v + 2] + 1
        return n, W, rp, ci, bits, "row pointers"
    raise ValueError(kind)


KINDS = ["asymmetric", "unsorted", "duplicate", "self-loop", "extra-bit", "missing-bit", "id-n", "id-negative",
         "bit-beyond-n", "rowptr-start", "rowptr-end", "rowptr-decreasing"]


@pytest.mark.parametrize("kind", KINDS)
def test_malformed_graph_is_rejected(kind):
    n, W, rp, ci, bits, text = break_graph(kind)
    print(f"[validate] malformed {kind} n={n}", flush=True)
    dg = upload(n, W, rp, ci, bits)
    with pytest.raises(lx.LexbfsError) as e:
        lx.validate(dg)
    assert e.value.code == EGRAPH and text in str(e.value), str(e.value)
    with pytest.raises(lx.LexbfsError) as e:
        lx.chordal_test(dg, flags=lx.LEXBFS_FLAG_VALIDATE)
    assert e.value.code == EGRAPH and text in str(e.value), str(e.value)
    good = [lx.DeviceGraph.from_host(g, DEV) for g in (gg.gnp(100, 0.05, 1), gg.subtree(300, 80, 6, 2))]
    with pytest.raises(lx.LexbfsError) as e:
        lx.chordal_test_batch(good[:1] + [dg] + good[1:], flags=lx.LEXBFS_FLAG_VALIDATE)
    assert e.value.code == EGRAPH and "graph 1:" in str(e.value), str(e.value)


def valid_graphs():
    return [gg.from_edges(1, []), gg.from_edges(2, [(0, 1)]), gg.from_edges(64, []),
            gg.from_edges(65, [(0, 64), (63, 64)]), gg.gnp(1000, 0.01, 3), gg.subtree(3000, 700, 8, 4),
            gg.plant(gg.subtree(2000, 500, 8, 5), 7, 6), gg.intervals(5000, 10, 7),
            gg.from_edges(130, [(a, b) for a in range(130) for b in range(a + 1, 130)])]


def test_valid_graphs_pass_and_results_match():
    graphs = valid_graphs() + [gg.config_single_large()[0]]
    for g in graphs:
        print(f"[validate] valid {g.name} n={g.n}", flush=True)
        dg = lx.DeviceGraph.from_host(g, DEV)
        lx.validate(dg)
        r = lx.chordal_test(dg, flags=lx.LEXBFS_FLAG_VALIDATE)
        ref = oracle.chordal_test(g)
        assert np.array_equal(r.order.cpu().numpy(), ref.order)
        assert r.chordal == ref.chordal and r.witness == ref.witness and r.cycle_list == ref.cycle.tolist()
    batch = [lx.DeviceGraph.from_host(g, DEV) for g in graphs]
    rs = lx.chordal_test_batch(batch, flags=lx.LEXBFS_FLAG_VALIDATE, outputs=True)
    for g, r in zip(graphs, rs):
        ref = oracle.chordal_test(g)
        assert np.array_equal(r.order.cpu().numpy(), ref.order)
        assert r.chordal == ref.chordal and r.witness == ref.witness and r.cycle_list == ref.cycle.tolist()


def test_full_split_graph_passes():
    g = gg.config_worst_steps()[1]
    print(f"[validate] split n={g.n}", flush=True)
    lx.validate(lx.DeviceGraph.from_host(g, DEV))


def test_plan_validates_at_creation():
    n, W, rp, ci, bits, _ = break_graph("asymmetric")
    dg = upload(n, W, rp, ci, bits)
    good = lx.DeviceGraph.from_host(gg.gnp(300, 0.02, 9), DEV)
    with pytest.raises(lx.LexbfsError) as e:
        lx.BatchPlan([good, good, dg], flags=lx.LEXBFS_FLAG_VALIDATE)
    assert e.value.code == EGRAPH and "graph 2:" in str(e.value)
    p = lx.BatchPlan([good, good], flags=lx.LEXBFS_FLAG_VALIDATE)
    p.launch()
    torch.cuda.synchronize()
    ref = oracle.chordal_test(gg.gnp(300, 0.02, 9))
    assert all(r.chordal == ref.chordal and r.witness == ref.witness for r in p.results())
    p.close()
