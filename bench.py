#!/usr/bin/env python3
"""Benchmark: chordality tests/s and edges/s, batched vs per-graph, on one MI355X.

Default workload (the batching configuration): 4,096 graphs with N
log-uniform on [32, 4096] -- 50% subtree-intersection chordal graphs, 25%
G(n, p) with average degree 8, 25% subtree graphs with a planted chordless
cycle of length 4..12 -- seed 0, synthetic, resident in HBM before timing.

A step is one pass of the whole path over the batch: one prepared
lexbfs_batch_plan_launch (LexBFS for every graph, the perfect-elimination
sweep, witnesses and certificates). `value` is whole-job tests/s over the K
timed steps. The per-graph path (one chordal_test call per graph) is timed
on an evenly spaced sample of the same graphs, and the CPU oracle on a
bounded sample on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch|single-small|single-large|split]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch",
                    choices=["batch", "single-small", "single-large", "split", "serving"])
    ap.add_argument("--serving-pool", type=int, default=192)
    ap.add_argument("--serving-requests", type=int, default=800)
    ap.add_argument("--per-graph-sample", type=int, default=512)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def pct(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else None


def algorithmic_bytes(graphs):
    """Per pass: the bitset read once (n rows of ceil(n/64) words) and the
    int32 per-vertex arrays each kernel touches."""
    bitset = sum(g.n * 8 * ((g.n + 63) // 64) for g in graphs)
    sn = sum(g.n for g in graphs)
    return {"lexbfs": bitset + 12 * sn,  # pivot rows; order, rank, parent written
            "sweep": bitset + 8 * sn,    # every row once; rank and parent read
            "certificate": 0, "setup": 0}


def roofline_from(timing, steps, graphs):
    """Algorithmic bytes of one pass split evenly over the launches of one
    pass (a batch pass launches each kernel once; the single-graph workloads
    launch each kernel once per graph, and their graphs have equal n)."""
    ab = algorithmic_bytes(graphs)
    per_kind = {}
    for kind, (count, ms) in timing.items():
        if count == 0:
            continue
        avg_s = ms / count / 1e3
        per_launch = ab.get(kind, 0) * steps / count
        per_kind[kind] = {"launches": count, "avg_ms": ms / count, "bytes_per_launch": per_launch,
                          "gbs": (per_launch / avg_s / 1e9) if avg_s > 0 else None}
    dom = max(per_kind, key=lambda k: timing[k][1])
    d = per_kind[dom]
    roof = {"bound": "hbm", "achieved": d["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (d["gbs"] / HBM_PEAK_GBS) if d["gbs"] is not None else None, "traffic": None,
            "kernel": dom, "avg_launch_ms": d["avg_ms"], "algorithmic_bytes_per_launch": d["bytes_per_launch"]}
    return roof, per_kind


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the chordality path here runs on a single MI355X "
              "(--gpus above 1 is not supported; see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen as gg
    import paper_1508_06329_amd as lx

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "serving":
        return bench_serving(args)
    t = time.time()
    if args.workload == "batch":
        graphs = gg.config_batch()
        wl = {"workload": "batch: 4,096 graphs, N log-uniform on [32, 4096], 50% subtree-intersection chordal / "
                          "25% G(n,p) avg degree 8 / 25% subtree + planted chordless cycle (length 4..12), seed 0"}
    elif args.workload == "single-small":
        graphs = gg.config_single_small()
        wl = {"workload": "single: N=1,024 subtree graph (tree 256, size [1,8]) and N=1,029 with a planted C5, seed 0"}
    elif args.workload == "single-large":
        graphs = gg.config_single_large()
        wl = {"workload": "single: N=16,384 subtree graph (tree 4,096, size [1,16]) and G(16384, 0.003), seed 0"}
    else:
        graphs = gg.config_worst_steps()
        wl = {"workload": "single: N=65,536 split graph (K=4,096 clique, 61,440 independent, 64 clique neighbours "
                          "each) and the copy minus one clique edge, seed 0"}
    sum_n = sum(g.n for g in graphs)
    sum_m = sum(g.m for g in graphs)
    log(f"generated {len(graphs)} graphs, sum N={sum_n}, sum M={sum_m} in {time.time() - t:.1f}s")
    dgs = lx.pack_graphs(graphs, dev)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    # ---------------- batched path ----------------
    if args.workload == "batch":
        plan = lx.BatchPlan(dgs)

        def step():
            plan.launch()
    else:
        ws = [torch.empty(lx.workspace_bytes(g.n), dtype=torch.uint8, device=dev) for g in dgs]
        res = torch.zeros((len(dgs), 8), dtype=torch.int32, device=dev)
        lib = lx._lib.load()
        descs = [g.desc() for g in dgs]
        import ctypes

        def step():
            for i, d in enumerate(descs):
                rc = lib.chordal_test(ctypes.byref(d), res[i].data_ptr(), None, ws[i].data_ptr(), ws[i].numel(), 0,
                                      stream.cuda_stream)
                lx._lib.check(rc, "chordal_test")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    with lx.KernelTimer() as kt:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            evs[k][0].record()
            step()
            evs[k][1].record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        timing = kt.collect()
    elapsed = t1 - t0
    step_ms = [a.elapsed_time(b) for a, b in evs]
    value = len(graphs) * args.steps / elapsed
    log(f"timed {args.steps} steps in {elapsed:.3f}s -> {value:.1f} tests/s")
    roof, per_kind = roofline_from(timing, args.steps, graphs)

    # ---------------- per-graph path ----------------
    per_graph = None
    if args.workload == "batch":
        idx = np.linspace(0, len(dgs) - 1, min(args.per_graph_sample, len(dgs))).astype(int)
        sample = [dgs[i] for i in idx]
        maxn = max(g.n for g in sample)
        ws1 = torch.empty(lx.workspace_bytes(maxn), dtype=torch.uint8, device=dev)
        res1 = torch.zeros(8, dtype=torch.int32, device=dev)
        lib = lx._lib.load()
        import ctypes

        descs = [g.desc() for g in sample]

        def one(d):
            rc = lib.chordal_test(ctypes.byref(d), res1.data_ptr(), None, ws1.data_ptr(), ws1.numel(), 0,
                                  stream.cuda_stream)
            lx._lib.check(rc, "chordal_test")

        for d in descs[:16]:
            one(d)
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for d in descs:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            one(d)
            b.record()
            lat.append((a, b))
        torch.cuda.synchronize()
        pg_elapsed = time.perf_counter() - t0
        lat_ms = [a.elapsed_time(b) for a, b in lat]
        pg_rate = len(descs) / pg_elapsed
        sm = sum(graphs[i].m for i in idx)
        per_graph = {"tests_per_s": pg_rate, "edges_per_s": sm / pg_elapsed, "sample_graphs": len(descs),
                     "latency_ms_p50": pct(lat_ms, 50), "latency_ms_p99": pct(lat_ms, 99),
                     "batched_speedup": value / pg_rate}
        log(f"per-graph path: {pg_rate:.1f} tests/s on {len(descs)} graphs")

    # ---------------- CPU oracle baseline ----------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        done, t0 = 0, time.perf_counter()
        edges = 0
        order = list(range(len(graphs)))
        while True:
            g = graphs[order[done % len(graphs)]]
            oracle.chordal_test(g)
            edges += g.m
            done += 1
            if time.perf_counter() - t0 >= args.cpu_seconds or done >= 4 * len(graphs):
                break
        cpu_el = time.perf_counter() - t0
        cpu = {"value": done / cpu_el, "unit": "tests/s", "cores": 1, "kind": "oracle",
               "sample": f"{done} graphs of the same workload in generation order ({cpu_el:.1f}s, one thread: "
                         f"partition-refinement LexBFS + parent test + certificate)",
               "edges_per_s": edges / cpu_el}
        log(f"cpu oracle: {cpu['value']:.1f} tests/s")

    out = {
        "metric": "chordality tests/s and edges/s, batched vs per-graph on 1 MI355X; p50/p99 ms",
        "value": value,
        "unit": "tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": dict(wl, graphs=len(graphs), sum_n=sum_n, sum_m=sum_m, parallelism="1 GPU"),
        "edges_per_s": sum_m * args.steps / elapsed,
        "step_ms_p50": pct(step_ms, 50),
        "step_ms_p99": pct(step_ms, 99),
        "roofline": roof,
        "kernels": per_kind,
        "per_graph": per_graph,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_serving(args):
    """Poisson stream of graphs, N log-uniform on [64, 32768], the 50/25/25
    mix, admitted under a 64 GB device budget. Requests replay a pool of
    distinct graphs (kept in page-locked host memory, uploaded per request).
    First the capacity (every request queued at t = 0), then offered rates
    of 0.5x and 0.8x that capacity for the continuous-batching server and
    for the plain per-graph path (one chordal_test per request, FIFO)."""
    import numpy as np

    import graphgen as gg
    from concurrent.futures import ThreadPoolExecutor
    from paper_1508_06329_amd import serving

    P, R = args.serving_pool, args.serving_requests
    t = time.time()
    ns, kinds, Ls, _ = gg.mix_specs(P, 64, 32768, 7)
    with ThreadPoolExecutor(max_workers=16) as ex:
        pool = list(ex.map(lambda i: gg.mix_graph(int(ns[i]), int(kinds[i]), int(Ls[i]), gg.graph_seed(7, 1000 + i)),
                           range(P)))
    for g in pool:
        g.pinned = serving.pin_graph(g)
    log(f"serving pool: {P} graphs, mean N={np.mean(ns):.0f}, max N={ns.max()}, built in {time.time() - t:.1f}s")
    rng = np.random.default_rng(0)
    pick = rng.integers(0, P, size=R)
    graphs = [pool[i] for i in pick]
    unit_gaps = rng.exponential(1.0, size=R)
    budget = 64 << 30
    serving.serve(graphs[:32], np.zeros(32), budget_bytes=budget)  # warm-up
    cap = serving.serve(graphs, np.zeros(R), budget_bytes=budget)
    log(f"capacity: {cap['throughput']:.0f} tests/s")
    rows = {}
    for frac in (0.5, 0.8):
        lam = frac * cap["throughput"]
        arr = np.cumsum(unit_gaps) / lam
        out = serving.serve(graphs, arr, budget_bytes=budget)
        rows[f"batched@{frac}"] = {k: out[k] for k in ("throughput", "p50_ms", "p99_ms", "peak_bytes")}
        rows[f"batched@{frac}"]["offered"] = lam
        log(f"batched at {lam:.0f}/s: {out['throughput']:.0f} tests/s p50 {out['p50_ms']:.2f} ms p99 {out['p99_ms']:.2f} ms")
    Rs = max(32, R // 4)
    lam = 0.5 * cap["throughput"]
    arr = np.cumsum(unit_gaps[:Rs]) / lam
    out = serving.serve(graphs[:Rs], arr, budget_bytes=budget, serial=True)
    rows["per_graph@0.5"] = {k: out[k] for k in ("throughput", "p50_ms", "p99_ms", "peak_bytes")}
    rows["per_graph@0.5"]["offered"] = lam
    log(f"per-graph at {lam:.0f}/s: {out['throughput']:.0f} tests/s p50 {out['p50_ms']:.2f} ms p99 {out['p99_ms']:.2f} ms")
    edges = float(np.mean([g.m for g in graphs]))
    main_row = rows["batched@0.8"]
    line = {
        "metric": "chordality tests/s and edges/s, batched vs per-graph on 1 MI355X; p50/p99 ms",
        "value": main_row["throughput"], "unit": "tests/s", "n_gpus": 1, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"serving: Poisson arrivals, N log-uniform on [64, 32768], 50/25/25 mix, "
                               f"{R} requests over a pool of {P} graphs, 64 GB admission budget, seed 0",
                   "parallelism": "1 GPU"},
        "capacity_tests_per_s": cap["throughput"], "edges_per_s": main_row["throughput"] * edges,
        "p50_ms": main_row["p50_ms"], "p99_ms": main_row["p99_ms"], "rates": rows,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
