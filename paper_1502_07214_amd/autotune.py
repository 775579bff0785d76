"""Launch-shape autotuner for the sweep kernels.

The shape (waves per walker, Philox blocks per lane, thresholds in LDS or read
through the caches) never changes results, only speed.  Candidates are timed
on throwaway clones of the job (same L, T, walker count, seed and weights) with
HIP events, so the job being tuned keeps its exact chain.  Choices can be kept
in a JSON cache keyed by device name and job shape.
"""
from __future__ import annotations

import json
import os
from typing import Optional, Sequence


from .muca import MucaBatch, MucaError, MucaJob

PLAIN_SHAPES = [(w, b, t) for w in (4, 2, 1) for b in (1, 2) for t in (1, 0)]
BATCH_SHAPES = [(w, b) for w in (0, 1, 2, 4) for b in (1, 2)]


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device())


def _load(cache: Optional[str]) -> dict:
    if cache and os.path.exists(cache):
        with open(cache) as f:
            return json.load(f)
    return {}


def _save(cache: Optional[str], data: dict):
    if cache:
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)


def _time(run, sweeps: int) -> float:
    import torch
    run(max(1, sweeps // 4))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    run(sweeps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def tune_job(L: int, T: float, n_walkers: int, seed: int = 0, lnW=None, probe_sweeps: int = 200,
             cache: Optional[str] = None) -> tuple:
    """Fastest (waves_per_walker, blocks_per_lane, lds_tables) for this job shape."""
    key = f"plain|{_device_name()}|L{L}|T{T!r}|W{n_walkers}"
    data = _load(cache)
    if key in data:
        return tuple(data[key]["shape"])
    best, best_ms, timings = None, float("inf"), {}
    for shape in PLAIN_SHAPES:
        clone = MucaJob(L, T, n_walkers, seed=seed, lnW=lnW, max_delta=1)
        try:
            clone.set_launch(*shape)
        except MucaError:
            clone.free()
            continue
        ms = _time(clone.sweep, probe_sweeps)
        clone.free()
        timings[str(shape)] = ms
        if ms < best_ms:
            best, best_ms = shape, ms
    data[key] = {"shape": list(best), "ms": best_ms, "probe_sweeps": probe_sweeps, "timings": timings}
    _save(cache, data)
    return best


def tune_batch(specs: Sequence[tuple], probe_sweeps: int = 100, cache: Optional[str] = None) -> tuple:
    """Fastest (waves_per_walker, blocks_per_lane) for a batch of jobs given as
    (L, T, n_walkers, seed) tuples."""
    sig = ",".join(f"{L}:{T!r}:{n}" for (L, T, n, _) in sorted(specs))
    key = f"batch|{_device_name()}|{sig}"
    data = _load(cache)
    if key in data:
        return tuple(data[key]["shape"])
    clones = [MucaJob(L, T, n, seed=s, max_delta=1) for (L, T, n, s) in specs]
    batch = MucaBatch(clones)
    best, best_ms, timings = None, float("inf"), {}
    for shape in BATCH_SHAPES:
        try:
            batch.set_launch(*shape)
        except MucaError:
            continue
        ms = _time(batch.sweep, probe_sweeps)
        timings[str(shape)] = ms
        if ms < best_ms:
            best, best_ms = shape, ms
    batch.free()
    for c in clones:
        c.free()
    data[key] = {"shape": list(best), "ms": best_ms, "probe_sweeps": probe_sweeps, "timings": timings}
    _save(cache, data)
    return best
