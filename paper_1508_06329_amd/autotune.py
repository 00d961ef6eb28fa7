"""Schedule autotuner for the batched launch.

The batch kernel runs each graph either on one 64-lane wavefront (four
graphs per workgroup, each in its own LDS region) or on a whole 256-lane
workgroup. Which is faster depends on the size mix: a wavefront team has no
workgroup barriers per step but owns four times as many vertices per lane,
and its LDS region caps how many graphs share a compute unit. The threshold
``wave_max_n`` (graphs with n <= threshold go to wavefronts) is chosen here
by timing one prepared launch per candidate on the caller's own graphs.

Candidate -1 is the all-workgroup schedule (block per graph); the others
mix wave-per-graph for small graphs with block-per-graph for the rest.
Results are cached per size signature for the life of the process.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import torch

DEFAULT_CANDIDATES = (-1, 128, 256, 384, 512, 768, 1024)

_cache: Dict[tuple, dict] = {}


def signature(graphs) -> tuple:
    """Graphs with the same sorted size list get the same schedule."""
    return tuple(sorted((g.n for g in graphs), reverse=True))


def time_plan(plan, reps: int, stream) -> float:
    """Median milliseconds of `reps` launches of a prepared plan."""
    plan.launch(stream=stream)
    stream.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.launch(stream=stream)
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    ms.sort()
    return ms[len(ms) // 2]


def autotune_batch(graphs: Sequence, candidates: Sequence[int] = DEFAULT_CANDIDATES, reps: int = 3,
                   stream: Optional[torch.cuda.Stream] = None, use_cache: bool = True, flags: int = 0) -> dict:
    """Time the batch launch over `graphs` (DeviceGraphs) for each candidate
    wave threshold and return ``{"tuning": {"wave_max_n": best}, "ms": {candidate: ms}}``.
    `flags` are the plan's flags (e.g. the MCS ordering).
    Candidates the plan rejects (their wavefront state does not fit LDS)
    are recorded as None."""
    from . import BatchPlan, LexbfsError

    key = (signature(graphs), tuple(candidates), flags)
    if use_cache and key in _cache:
        return _cache[key]
    stream = stream or torch.cuda.current_stream()
    table = {}
    for c in candidates:
        try:
            plan = BatchPlan(graphs, tuning={"wave_max_n": c}, stream=stream, flags=flags)
        except LexbfsError:
            table[c] = None
            continue
        try:
            table[c] = time_plan(plan, reps, stream)
        finally:
            stream.synchronize()
            plan.close()
    timed = {c: t for c, t in table.items() if t is not None}
    if not timed:
        raise RuntimeError("no candidate schedule could be prepared for these graphs")
    best = min(timed, key=timed.get)
    out = {"tuning": {"wave_max_n": best}, "ms": table}
    _cache[key] = out
    return out
