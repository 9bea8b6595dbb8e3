"""Project autotuner for batched tracking launches.

A batch's launch plan (poses per scoring workgroup, persistent scoring grid, item order) is chosen
per shape class by timing every candidate on the device with HIP events around
`track_batch_run`. Results are stored in a JSON table keyed by the shape class, which
`plan_for` consults. Every candidate computes the same result bit for bit (the per-pose reduction
order does not depend on the plan), so tuning trades nothing for speed.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Dict, Iterable, List, Optional, Sequence

from . import BatchPlan, Batch

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_table.json")

CANDIDATES: List[BatchPlan] = [BatchPlan(tk, grid, order)
                               for tk in (0, 1, 2, 4, 8) for grid in (128, 256, 512, 1024, 2048, 4096)
                               for order in (0, 1)]


def shape_class(problems) -> str:
    """Coarse key of a batch: problem count, format/layout, and log2 buckets of the summed
    particle-point work and of the mean particle count."""
    import math
    n = len(problems)
    work = sum(p[2].width * p[2].height * (p[5].K + 1) / (p[5].pixel_stride ** 2) for p in problems)
    kmean = sum(p[5].K for p in problems) / n
    vol = problems[0][0]
    return f"n{n}-f{vol.format}-l{vol.layout}-w{int(math.log2(max(work, 1)))}-k{int(math.log2(max(kmean, 1)))}"


def load_table(path: str = TABLE) -> Dict[str, dict]:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def plan_for(problems, path: str = TABLE) -> BatchPlan:
    """The tuned plan of this batch's shape class, or the default plan."""
    entry = load_table(path).get(shape_class(problems))
    if entry is None:
        return BatchPlan()
    return BatchPlan(entry["score_tk"], entry["score_grid"], entry["order"])


def time_plan(problems, plan: BatchPlan, reps: int = 3, device="cuda") -> float:
    """Median ms of track_batch_run for `plan` (after one warm-up run)."""
    import torch
    b = Batch(problems, plan, device=device)
    try:
        b.run()
        torch.cuda.synchronize()
        times = []
        s = torch.cuda.current_stream()
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            b.run()
            e1.record(s)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        return sorted(times)[len(times) // 2]
    finally:
        b.close()


def tune(problems, candidates: Optional[Sequence[BatchPlan]] = None, reps: int = 3, path: Optional[str] = TABLE,
         log=print) -> BatchPlan:
    """Times every candidate plan on this batch and records the fastest for its shape class."""
    cands = list(candidates or CANDIDATES)
    results = []
    for c in cands:
        ms = time_plan(problems, c, reps)
        results.append((ms, c))
        if log:
            log(f"[autotune] tk={c.score_tk} grid={c.score_grid} order={c.order}: {ms:.3f} ms")
    ms, best = min(results, key=lambda r: r[0])
    if path:
        table = load_table(path)
        table[shape_class(problems)] = dict(dataclasses.asdict(best), ms=ms,
                                            worst_ms=max(r[0] for r in results))
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best
