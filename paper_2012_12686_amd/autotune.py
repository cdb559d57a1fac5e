"""Autotuner of the workgroup split per probe size.

For each probe size present in a set of jobs it times the persistent batched
launch of those jobs with every supported split (HIP events on the current
stream), keeps the fastest, and sets it on the context so later plans use it.
Results are cached in a JSON file keyed by the device, the probe size and the
shape of the work (positions and mean depth, bucketed).
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional

import torch

from .api import Context, Job

SPLITS = {64: (1, 2, 4), 96: (1, 2, 3, 4), 128: (1, 2, 4, 8), 192: (2, 4, 6, 8)}


def _key(device_name: str, n: int, jobs: List[Job]) -> str:
    pos = sum(int(j.corner.shape[0]) for j in jobs)
    depth = sum(j.geom.n_slices * int(j.corner.shape[0]) for j in jobs) / max(pos, 1)
    return f"{device_name}|N{n}|P{2 ** round(math.log2(max(pos, 1)))}|S{2 ** round(math.log2(max(depth, 1)))}"


def _time_plan(ctx: Context, jobs: List[Job], reps: int) -> float:
    plan = ctx.plan(jobs)
    try:
        plan.run()
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            plan.run()
        end.record()
        torch.cuda.synchronize()
        ctx.sync_error()
        return start.elapsed_time(end) / reps
    finally:
        plan.close()


def autotune(ctx: Context, jobs: List[Job], reps: int = 2, cache_path: Optional[str] = None) -> Dict[int, dict]:
    """Pick and set the best split for every probe size among ``jobs``.

    Returns {N: {"split": k, "ms": {k: milliseconds, ...}, "cached": bool}}.
    """
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
    dev_name = torch.cuda.get_device_name(ctx.device)
    result = {}
    for n in sorted({j.geom.n for j in jobs}):
        group = [j for j in jobs if j.geom.n == n]
        key = _key(dev_name, n, group)
        if key in cache:
            ctx.set_split(n, cache[key]["split"])
            result[n] = dict(cache[key], cached=True)
            continue
        times = {}
        for k in SPLITS[n]:
            ctx.set_split(n, k)
            times[k] = _time_plan(ctx, group, reps)
        best = min(times, key=times.get)
        ctx.set_split(n, best)
        result[n] = {"split": best, "ms": times, "cached": False}
        cache[key] = {"split": best, "ms": times}
    if cache_path:
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return result
