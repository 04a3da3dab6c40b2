"""Launch-schedule autotuning for the blend kernels.

The schedule (waves per workgroup, tile order, persistent tile queue) changes
only the order in which tiles are issued, never a result, so it is chosen by
timing: tune()
runs forward + backward under each candidate on the caller's own batch and
keeps the fastest.  Winners are cached per workload shape in a JSON file so
that later runs of the same shape skip the timing.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, Optional, Tuple

import torch

from . import render

# (waves per workgroup, tile order, persistent): tile order 0 row-major, 1
# XCD-grouped, 2 heaviest first; persistent 1 runs the blends as a resident
# grid that takes tiles from a queue in that order (one wave per workgroup)
CANDIDATES: Tuple[Tuple[int, int, int], ...] = ((1, 0, 0), (2, 0, 0), (4, 0, 0), (1, 1, 0), (1, 2, 0), (2, 2, 0),
                                                (4, 2, 0), (1, 0, 1), (1, 2, 1))


def default_cache_path() -> str:
    return os.environ.get("CGS_SCHEDULE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "cgs", "schedule.json"))


def shape_key(r: render.Renderer) -> str:
    """Views, log2 buckets of pixels and Gaussians, codebook dtype and SH degree."""
    n_g = sum(r.scenes[v].n for v in r.view_scene)
    s0 = r.scenes[0]
    dt = "bf16" if s0.descriptor().sr.dtype == 1 else "f32"
    return (f"v{len(r.cameras)}_p{int(math.log2(max(r.n_pixels, 1)))}"
            f"_g{int(math.log2(max(n_g, 1)))}_{dt}_d{s0.sh_degree}")


def _load(path: str) -> Dict[str, list]:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: str, data: Dict[str, list]) -> None:
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only costs the next run a re-tune


def time_schedule(r: render.Renderer, grad_image: torch.Tensor, reps: int) -> float:
    """Median milliseconds of one forward + backward on the current stream."""
    r.forward()
    r.backward(grad_image)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        r.forward()
        r.backward(grad_image)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tune(r: render.Renderer, grad_image: Optional[torch.Tensor] = None, reps: int = 5,
         candidates: Iterable[Tuple[int, int, int]] = CANDIDATES, cache_path: Optional[str] = None,
         use_cache: bool = True) -> Tuple[Tuple[int, int, int], Dict[str, float]]:
    """Pick the fastest schedule for this renderer's batch and apply it.
    Returns ((waves_per_block, tile_order, persistent), {candidate: ms}); the
    timings are empty when the cache answered."""
    path = cache_path or default_cache_path()
    key = shape_key(r)
    cache = _load(path) if use_cache else {}
    hit = cache.get(key)
    candidates = tuple(tuple(c) for c in candidates)
    if hit and tuple(hit) in set(candidates):
        r.set_schedule(*hit)
        return tuple(int(x) for x in hit), {}
    if grad_image is None:
        grad_image = torch.full((r.n_pixels, 3), 1e-6, dtype=torch.float32, device=r.device)
    timings: Dict[str, float] = {}
    best, best_ms = None, float("inf")
    for cand in candidates:
        r.set_schedule(*cand)
        ms = time_schedule(r, grad_image, reps)
        timings[",".join(str(x) for x in cand)] = round(ms, 4)
        if ms < best_ms:
            best, best_ms = cand, ms
    r.set_schedule(*best)
    if use_cache:
        cache = _load(path)
        cache[key] = list(best)
        _store(path, cache)
    return best, timings
