"""Serving: continuous batching of chordality requests on one GPU.

Requests (graphs of mixed sizes) arrive over time. The server admits a
request when its device footprint (bitset + CSR + per-graph workspace) fits
the remaining memory budget and an in-flight slot is free, uploads it on a
copy stream, and folds every uploaded request that is not yet running into
the next batch launch. Launches go round-robin over several compute
streams, so a batch formed while earlier ones still run overlaps them on the
device. When a launch completes, its requests record their latency
(completion - arrival) and release their memory, which admits more.

Every admitted graph goes into the launch's batch plan; graphs above the
256-lane tier's size run on their own 1024-lane workgroups inside the same
launch (on the plan's side stream), concurrently with the rest. Every result
is a pure function of its own graph, so a request gets the same verdict,
witness and certificate alone or in any mix.

The admission logic (:class:`AdmissionController`) is plain host code with no
device dependency; the tests drive it with a fake clock and executor.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional, Sequence

def footprint_bytes(n: int, nnz: int, W: Optional[int] = None) -> int:
    """Device bytes one request holds while admitted: the bitset, the CSR,
    its result record and its share of the workspace (about ten int32
    arrays of n entries, 256-byte aligned)."""
    W = (n + 63) // 64 if W is None else W
    al = lambda x: (x + 255) // 256 * 256
    return al(8 * max(n * W, 1)) + al(4 * (n + 1)) + al(4 * max(nnz, 1)) + 10 * al(4 * max(n, 1)) + 1024


@dataclass
class Request:
    rid: int
    graph: object                 # host graph (graphgen.Graph-like)
    arrival: float                # seconds, on the server's clock
    nbytes: int = 0
    admitted: float = -1.0
    done: float = -1.0
    result: object = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class AdmissionController:
    """FIFO admission under a byte budget and a slot limit.

    A request larger than the whole budget can never be admitted; it is
    rejected (``rejected``) instead of blocking the queue."""

    def __init__(self, budget_bytes: int, max_inflight: int = 1 << 30):
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        self.used = 0
        self.inflight = 0
        self.queue: Deque[Request] = collections.deque()
        self.rejected: List[Request] = []
        self.peak_used = 0

    def submit(self, r: Request):
        if r.nbytes > self.budget:
            self.rejected.append(r)
        else:
            self.queue.append(r)

    def admit(self, now: float) -> List[Request]:
        """Admit from the head of the queue while the head fits."""
        out = []
        while self.queue and self.inflight < self.max_inflight and self.used + self.queue[0].nbytes <= self.budget:
            r = self.queue.popleft()
            self.used += r.nbytes
            self.inflight += 1
            r.admitted = now
            out.append(r)
        self.peak_used = max(self.peak_used, self.used)
        return out

    def release(self, r: Request):
        self.used -= r.nbytes
        self.inflight -= 1
        assert self.used >= 0 and self.inflight >= 0


def run_loop(requests: Sequence[Request], ctrl: AdmissionController, executor, clock: Callable[[], float],
             idle: Callable[[], None], max_launches=3, classify: Optional[Callable[[Request], object]] = None):
    """Drive arrivals, admission, launches and completions until every
    request is done or rejected.

    Admitted requests wait in the queue of their class (``classify(r)``; a
    single class if None). A class launches all its waiting requests at once
    whenever fewer than its limit of its launches are running
    (``max_launches``: an int for every class, or a dict class -> limit), so
    requests arriving meanwhile are folded into its next launch. `executor`
    provides ``start(requests[, cls]) -> handle`` (upload + launch,
    asynchronous; cls passed only when classify is given),
    ``ready(handle) -> bool`` and ``finish(handle)`` (collect results).
    Returns the requests in completion order."""
    limit = (lambda c: max_launches.get(c, 1)) if isinstance(max_launches, dict) else (lambda c: max_launches)
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    waiting: Dict[object, List[Request]] = collections.defaultdict(list)
    inflight: Dict[object, int] = collections.defaultdict(int)
    running = []
    finished = []
    total = len(requests)
    while len(finished) + len(ctrl.rejected) < total:
        now = clock()
        while pending and pending[0].arrival <= now:
            ctrl.submit(pending.popleft())
        progressed = False
        for r in ctrl.admit(now):
            waiting[classify(r) if classify else None].append(r)
        for c, rs in waiting.items():
            if rs and inflight[c] < limit(c):
                h = executor.start(rs, c) if classify else executor.start(rs)
                running.append((h, rs, c))
                inflight[c] += 1
                waiting[c] = []
                progressed = True
        still = []
        for h, rs, c in running:
            if executor.ready(h):
                executor.finish(h)
                t = clock()
                for r in rs:
                    r.done = t
                    ctrl.release(r)
                    finished.append(r)
                inflight[c] -= 1
                progressed = True
            else:
                still.append((h, rs, c))
        running = still
        if not progressed:
            idle()
    return finished


def percentile(xs: Sequence[float], q: float) -> float:
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def pin_graph(g):
    """Page-locked host copies (row_ptr, col_idx, bits) of a host graph, so
    its upload is a plain asynchronous DMA."""
    import torch

    ci = g.col_idx if g.col_idx.size else g.col_idx.reshape(0)
    return (torch.from_numpy(g.row_ptr).pin_memory(), torch.from_numpy(ci).pin_memory(),
            torch.from_numpy(g.bits.view("int64")).pin_memory())


# Requests up to this size form the short class: their launches end within
# a few milliseconds and never wait for a long graph's chain.
SHORT_MAX_N = 4096


class GpuExecutor:
    """Uploads admitted graphs on a copy stream and launches each class's
    batch as one prepared plan on the next of that class's compute streams.
    Classes: short (n <= SHORT_MAX_N), mid (up to the 256-lane tier's limit)
    and long (the 1024-lane tier), so a launch lasts only as long as the
    longest chain of its own class."""

    def __init__(self, device="cuda", streams: Optional[Dict[str, int]] = None, outputs: bool = False):
        import torch

        from . import _lib

        self.torch = torch
        self.lib = _lib.load()
        self.dev = torch.device(device)
        self.copy = torch.cuda.Stream(device=self.dev)
        counts = streams or {"short": 1, "mid": 1, "long": 2}
        self.streams = {c: [torch.cuda.Stream(device=self.dev) for _ in range(k)] for c, k in counts.items()}
        self.next = {c: 0 for c in counts}
        self.launch_limits = dict(counts)
        self.outputs = outputs
        tier = int(self.lib.lexbfs_batch_max_n())
        _lib.check(min(tier, 0), "lexbfs_batch_max_n")
        self.tier_max = tier

    def classify(self, r: Request) -> str:
        n = r.graph.n
        if "mid" not in self.streams:
            return next(iter(self.streams))
        return "short" if n <= SHORT_MAX_N else "mid" if n <= self.tier_max else "long"

    def _upload(self, graphs):
        from . import DeviceGraph

        torch = self.torch
        out = []
        with torch.cuda.stream(self.copy):
            for g in graphs:
                hp = getattr(g, "pinned", None) or pin_graph(g)
                rp, ci, bits = (t.to(self.dev, non_blocking=True) for t in hp)
                out.append(DeviceGraph(g.n, g.W, rp, ci, bits))
        ev = torch.cuda.Event()
        ev.record(self.copy)
        return out, ev

    def start(self, reqs: Sequence[Request], cls: str = "short"):
        from . import BatchPlan

        torch = self.torch
        group = self.streams[cls]
        s = group[self.next[cls] % len(group)]
        self.next[cls] += 1
        dgs, _ = self._upload([r.graph for r in reqs])
        # The plan stages its descriptor table on the copy stream, behind the
        # uploads only, so preparing it never waits for a running launch.
        with torch.cuda.stream(self.copy):
            plan = BatchPlan(dgs, outputs=self.outputs, stream=self.copy)
        ready = torch.cuda.Event()
        ready.record(self.copy)
        s.wait_event(ready)
        handle = {"stream": s, "reqs": reqs, "dgs": dgs, "plan": plan, "singles": []}
        with torch.cuda.stream(s):
            plan.launch(stream=s)
        ev = torch.cuda.Event()
        ev.record(s)
        handle["event"] = ev
        return handle

    def ready(self, handle) -> bool:
        return handle["event"].query()

    def finish(self, handle):
        from . import Result, _result_from

        reqs = handle["reqs"]
        if handle["plan"] is not None:
            for r, res in zip(reqs, handle["plan"].results()):
                r.result = res
            handle["plan"].close()
        for i, res, ws, tens in handle["singles"]:
            chordal, wit, clen, fb = _result_from(res.cpu())
            n = handle["dgs"][i].n
            reqs[i].result = Result(chordal, wit, clen, fb, **{k: v[:n] for k, v in tens.items()})
        handle["dgs"] = None


class SerialExecutor(GpuExecutor):
    """The plain per-graph path: one request at a time, one chordal_test per
    request, on one stream (admission limited to one in flight)."""

    def __init__(self, device="cuda", outputs: bool = False):
        super().__init__(device, streams={"all": 1}, outputs=outputs)

    def start(self, reqs: Sequence[Request], cls: str = "all"):
        from . import _lib, _zeros_on, lexbfs_outputs_t

        torch = self.torch
        s = self.streams["all"][0]
        dgs, up = self._upload([r.graph for r in reqs])
        s.wait_event(up)
        handle = {"stream": s, "reqs": reqs, "dgs": dgs, "plan": None, "singles": []}
        for i, g in enumerate(dgs):
            res = _zeros_on(8, self.dev, s)  # the fill runs on s, ahead of the test
            outs = lexbfs_outputs_t()
            tens = {}
            if self.outputs:
                for k in ("order", "rank", "parent", "cycle"):
                    tens[k] = torch.empty(max(g.n, 1), dtype=torch.int32, device=self.dev)
                    setattr(outs, k, tens[k].data_ptr())
            ws = torch.empty(self.lib.lexbfs_workspace_bytes(g.n), dtype=torch.uint8, device=self.dev)
            d = g.desc()
            rc = self.lib.chordal_test(ctypes.byref(d), res.data_ptr(), ctypes.byref(outs), ws.data_ptr(),
                                       ws.numel(), 0, s.cuda_stream)
            _lib.check(rc, "chordal_test")
            handle["singles"].append((i, res, ws, tens))
        ev = torch.cuda.Event()
        ev.record(s)
        handle["event"] = ev
        return handle


def serve(graphs: Sequence, arrivals: Sequence[float], budget_bytes: int = 64 << 30, serial: bool = False,
          outputs: bool = False, max_inflight: int = 1 << 30, device="cuda") -> Dict:
    """Run a request stream (graphs[i] arrives at arrivals[i] seconds after
    the start) through the continuous-batching server (or, with
    serial=True, through the plain per-graph path). Returns the requests
    and summary statistics."""
    ex = SerialExecutor(device, outputs) if serial else GpuExecutor(device, outputs=outputs)
    ctrl = AdmissionController(budget_bytes, 1 if serial else max_inflight)
    reqs = [Request(i, g, float(a), footprint_bytes(g.n, g.nnz, g.W)) for i, (g, a) in enumerate(zip(graphs, arrivals))]
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    done = run_loop(reqs, ctrl, ex, clock, idle=lambda: time.sleep(20e-6), max_launches=ex.launch_limits,
                    classify=ex.classify)
    wall = clock()
    lat = [r.latency for r in done]
    span = max(r.done for r in done) - min(r.arrival for r in done) if done else float("nan")
    return {
        "requests": reqs,
        "completed": len(done),
        "rejected": len(ctrl.rejected),
        "wall_s": wall,
        "throughput": len(done) / span if span > 0 else float("nan"),
        "p50_ms": percentile(lat, 50) * 1e3,
        "p99_ms": percentile(lat, 99) * 1e3,
        "peak_bytes": ctrl.peak_used,
    }
