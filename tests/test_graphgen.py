"""The seeded input generators: format invariants and the shapes the
workloads ask for. (Inputs only; the chordality arithmetic is tested
elsewhere.)"""
import math

import numpy as np
import pytest

import graphgen as gg
from brute import chordal_by_elimination


def check_format(g):
    n, W = g.n, g.W
    B = g.bits.reshape(n, W) if n else g.bits.reshape(0, W)
    # padding bits beyond n are zero
    if n % 64 and n:
        pad = ~np.uint64((1 << (n % 64)) - 1)
        assert not (B[:, (n - 1) // 64] & pad).any()
    assert not B[:, (n + 63) // 64:].any()
    # CSR ascending, no self loops, matches the bitset, symmetric
    rp, ci = g.row_ptr, g.col_idx
    assert rp[0] == 0 and rp[-1] == ci.size
    src = np.repeat(np.arange(n), np.diff(rp))
    assert (src != ci).all()
    for v in range(0, n, max(1, n // 97)):
        row = g.neighbors(v)
        assert (np.diff(row) > 0).all()
        bits_row = np.unpackbits(B[v].view(np.uint8), bitorder="little")[:n]
        assert np.array_equal(np.nonzero(bits_row)[0], row)
    key = src.astype(np.int64) * n + ci
    rkey = ci.astype(np.int64) * n + src
    assert np.array_equal(np.sort(key), np.sort(rkey))


def test_splitmix64_published_vector():
    # SplitMix64 from state 0 (the widely published reference output)
    assert gg.splitmix_stream(0, 3).tolist() == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_rng_deterministic_and_uniform():
    a = gg.rng_stream(42, 20000)
    b = gg.rng_stream(42, 20000)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, gg.rng_stream(43, 20000))
    bits = np.unpackbits(a.view(np.uint8))
    assert abs(bits.mean() - 0.5) < 0.01


@pytest.mark.parametrize("n,T,s", [(1, 1, 1), (50, 10, 4), (300, 64, 8), (1000, 256, 8)])
def test_subtree_format_and_chordal(n, T, s):
    g = gg.subtree(n, T, s, gg.graph_seed(5, n))
    check_format(g)
    if n <= 50:
        assert chordal_by_elimination(n, g.adj_sets())


def test_gnp_density():
    g = gg.gnp(3000, 0.01, 9)
    check_format(g)
    exp = 3000 * 2999 / 2 * 0.01
    assert abs(g.m - exp) < 5 * math.sqrt(exp)


def test_split_shape():
    K, I, a = 50, 400, 7
    g = gg.split(K, I, a, 3)
    check_format(g)
    deg = np.diff(g.row_ptr)
    assert (deg[K:] == a).all()
    assert (g.col_idx[g.row_ptr[K]:] < K).all()
    assert g.m == K * (K - 1) // 2 + I * a
    h0, h1 = gg.split_pair(K, I, a, 3)
    assert h1.m == h0.m - 1
    a0, b0 = h1.meta["removed"]
    assert not h1.has_edge(a0, b0) and h0.has_edge(a0, b0)


def test_plant_adds_cycle_and_bridge():
    g = gg.subtree(100, 30, 5, 1)
    h = gg.plant(g, 7, 2)
    check_format(h)
    assert h.n == 107 and h.m == g.m + 8
    for i in range(7):
        assert h.has_edge(100 + i, 100 + (i + 1) % 7)
    bridge = [u for u in h.neighbors(100) if u < 100]
    assert len(bridge) == 1


def test_workload_small_shapes():
    g, h = gg.config_single_small()
    assert (g.n, h.n) == (1024, 1029)
    check_format(g)
    check_format(h)
    assert h.m == g.m + 6


def test_mix_specs():
    ns, kinds, Ls, gaps = gg.mix_specs(4096, 32, 4096, 0)
    assert ns.min() >= 32 and ns.max() <= 4096
    assert (kinds == 0).sum() == 2048 and (kinds == 1).sum() == 1024 and (kinds == 2).sum() == 1024
    assert Ls.min() >= 4 and Ls.max() <= 12
    # log-uniform: median near sqrt(32 * 4097)
    assert abs(np.log(np.median(ns)) - 0.5 * np.log(32 * 4097)) < 0.15
    assert abs(gaps.mean() - 1.0) < 0.1


def test_batch_small_sample_formats():
    gs = gg.config_batch(count=24, lo=32, hi=300, seed=3)
    assert len(gs) == 24
    for g in gs:
        check_format(g)
