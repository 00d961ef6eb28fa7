"""Admission and the serving loop, on the host only: a fake clock and a fake
executor whose launches complete after a scripted delay, out of order."""
import random

import pytest

from paper_1508_06329_amd.serving import AdmissionController, Request, footprint_bytes, percentile, run_loop


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def idle(self):
        self.t += 1e-4


class FakeExecutor:
    """A launch of k requests finishes `dur(k)` after it starts."""

    def __init__(self, clock, dur, ctrl):
        self.clock, self.dur, self.ctrl = clock, dur, ctrl
        self.launches = []
        self.max_used = 0

    def start(self, reqs):
        self.max_used = max(self.max_used, self.ctrl.used)
        h = {"end": self.clock() + self.dur(reqs), "reqs": list(reqs)}
        self.launches.append(h)
        return h

    def ready(self, h):
        return self.clock() >= h["end"]

    def finish(self, h):
        for r in h["reqs"]:
            r.result = ("ok", r.rid)


def make_requests(n, rng, size_range=(1, 100), rate=1000.0):
    t = 0.0
    out = []
    for i in range(n):
        t += rng.expovariate(rate)
        out.append(Request(i, None, t, nbytes=rng.randint(*size_range)))
    return out


def test_footprint_grows_with_size():
    assert footprint_bytes(1000, 5000) < footprint_bytes(2000, 5000) < footprint_bytes(2000, 50000)
    assert footprint_bytes(65536, 0) >= 65536 * 1024 * 8


@pytest.mark.parametrize("seed", range(5))
def test_budget_never_exceeded_and_all_complete(seed):
    rng = random.Random(seed)
    reqs = make_requests(300, rng)
    ctrl = AdmissionController(budget_bytes=400, max_inflight=16)
    clk = FakeClock()
    ex = FakeExecutor(clk, lambda rs: 1e-3 * rng.random() * len(rs), ctrl)
    done = run_loop(reqs, ctrl, ex, clk, clk.idle)
    assert len(done) == 300 and not ctrl.rejected
    assert ctrl.peak_used <= 400 and ex.max_used <= 400
    assert ctrl.used == 0 and ctrl.inflight == 0
    assert all(r.result == ("ok", r.rid) for r in reqs)
    assert all(r.arrival <= r.admitted <= r.done for r in reqs)
    # FIFO admission
    adm = sorted(reqs, key=lambda r: (r.admitted, r.rid))
    assert [r.rid for r in adm] == sorted(r.rid for r in reqs)


def test_out_of_order_completion_releases_memory():
    ctrl = AdmissionController(budget_bytes=100)
    clk = FakeClock()
    # the first launch is slow, later ones fast: completions come out of order
    durs = iter([5e-2] + [1e-3] * 100)
    ex = FakeExecutor(clk, lambda rs: next(durs), ctrl)
    reqs = [Request(i, None, i * 1e-3, nbytes=30) for i in range(12)]
    done = run_loop(reqs, ctrl, ex, clk, clk.idle)
    assert len(done) == 12
    assert done[-1].rid == 0 or any(d.rid == 0 for d in done)
    assert [d.rid for d in done] != sorted(d.rid for d in done)  # not FIFO completion


def test_oversize_request_is_rejected_not_blocking():
    ctrl = AdmissionController(budget_bytes=50)
    clk = FakeClock()
    ex = FakeExecutor(clk, lambda rs: 1e-3, ctrl)
    reqs = [Request(0, None, 0.0, 10), Request(1, None, 0.0, 500), Request(2, None, 0.0, 10)]
    done = run_loop(reqs, ctrl, ex, clk, clk.idle)
    assert [r.rid for r in ctrl.rejected] == [1]
    assert sorted(r.rid for r in done) == [0, 2]


def test_slot_limit_serializes():
    ctrl = AdmissionController(budget_bytes=10 ** 9, max_inflight=1)
    clk = FakeClock()
    ex = FakeExecutor(clk, lambda rs: 1e-3, ctrl)
    reqs = [Request(i, None, 0.0, 1) for i in range(10)]
    run_loop(reqs, ctrl, ex, clk, clk.idle)
    assert all(len(h["reqs"]) == 1 for h in ex.launches)


def test_continuous_batching_groups_arrivals():
    # arrivals during a running launch are folded into the next launch
    ctrl = AdmissionController(budget_bytes=10 ** 9, max_inflight=10 ** 6)
    clk = FakeClock()
    ex = FakeExecutor(clk, lambda rs: 1e-2, ctrl)
    reqs = [Request(i, None, i * 1e-3, 1) for i in range(40)]
    run_loop(reqs, ctrl, ex, clk, clk.idle, max_launches=2)
    assert max(len(h["reqs"]) for h in ex.launches) > 1
    assert len(ex.launches) < 40
    # two launches overlap in time
    spans = sorted((h["end"] - 1e-2, h["end"]) for h in ex.launches)
    assert any(b[0] < a[1] for a, b in zip(spans, spans[1:]))


def test_percentile():
    xs = list(range(101))
    assert percentile(xs, 50) == 50 and percentile(xs, 99) == 99 and percentile(xs, 0) == 0


class ClassExecutor(FakeExecutor):
    def start(self, reqs, cls):
        h = super().start(reqs)
        h["cls"] = cls
        return h


def test_size_classes_do_not_wait_for_each_other():
    # long requests take 50 ms per launch, short ones 1 ms; with one launch
    # slot per class, short requests keep flowing while a long launch runs
    ctrl = AdmissionController(budget_bytes=10 ** 9)
    clk = FakeClock()
    ex = ClassExecutor(clk, lambda rs: 5e-2 if rs[0].nbytes > 50 else 1e-3, ctrl)
    reqs = [Request(i, None, i * 2e-3, 100 if i % 10 == 0 else 1) for i in range(60)]
    done = run_loop(reqs, ctrl, ex, clk, clk.idle, max_launches={"short": 1, "long": 1},
                    classify=lambda r: "long" if r.nbytes > 50 else "short")
    assert len(done) == 60
    assert all(h["cls"] == ("long" if h["reqs"][0].nbytes > 50 else "short") for h in ex.launches)
    assert all(len({r.nbytes > 50 for r in h["reqs"]}) == 1 for h in ex.launches)  # no mixed launch
    short_lat = sorted(r.latency for r in reqs if r.nbytes == 1)
    assert short_lat[len(short_lat) // 2] < 1e-2  # median short latency far below one long launch
    # a short launch overlaps a long one
    spans = [(h["end"] - (5e-2 if h["cls"] == "long" else 1e-3), h["end"], h["cls"]) for h in ex.launches]
    longs = [sp for sp in spans if sp[2] == "long"]
    assert any(a[0] < b[0] < a[1] for a in longs for b in spans if b[2] == "short")
