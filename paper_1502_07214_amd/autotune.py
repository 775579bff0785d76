"""Launch-shape autotuner for the sweep kernels.

The shape (waves per walker, Philox blocks per lane, thresholds in LDS or read
through the caches) never changes results, only speed.  Candidates are timed
on throwaway clones of the job (same L, T, walker count, seed and weights) with
HIP events, so the job being tuned keeps its exact chain.  Choices are kept in
a JSON cache keyed by device name and job shape; CACHE is the one the
benchmark uses, committed with the choices measured on an MI355X.
"""
from __future__ import annotations

import json
import os
from typing import Optional, Sequence


from .muca import MucaBatch, MucaError, MucaJob

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

# (waves per walker, Philox blocks per lane, thresholds in LDS, packed lattices)
PLAIN_SHAPES = [(w, b, t, p) for w in (4, 2, 1) for b in (1, 2) for t in (1, 0) for p in (0, 1) if b == 1 or p == 0]
# (waves per walker, Philox blocks per lane, persistent blocks (0: as many as
# fit on the device), packed lattices)
BATCH_SHAPES = [(w, b, 0, p) for w in (0, 1, 2, 4) for b in (1, 2) for p in (0, 1) if b == 1 or p == 0]


def batch_shapes(n_cu: int) -> list:
    """BATCH_SHAPES, each also with two persistent blocks per compute unit:
    fewer blocks than fit leave the long walkers of the largest lattices
    fewer waves to share their SIMDs with."""
    return [s for s in BATCH_SHAPES] + [(w, b, 2 * n_cu, p) for (w, b, _, p) in BATCH_SHAPES]


def _device_name() -> str:
    """The device's architecture and compute-unit count (the marketing name
    is not always available)."""
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "") or torch.cuda.get_device_name(torch.cuda.current_device())
    return f"{arch.split(':')[0]}/{p.multi_processor_count}cu"


def _warm(master: MucaJob, iterations: int, sweeps: int):
    """A few multicanonical iterations, so that shapes are timed on the
    weights and lattices of a running job rather than on the first sweeps
    from random lattices."""
    for _ in range(iterations):
        master.sweep(sweeps)
        master.update_weights(master.reduce_hist())


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
             cache: Optional[str] = None, shapes=None, warm: tuple = (0, 0)) -> tuple:
    """Fastest (waves_per_walker, blocks_per_lane, lds_tables, packing) for
    this job shape (from the cache when it holds one).  warm = (iterations, sweeps):
    the clones start from the state and weights of a master job taken through
    that many iterations first.  ValueError if no candidate shape is valid."""
    key = f"plain2|{_device_name()}|L{L}|T{T!r}|W{n_walkers}|warm{warm[0]}x{warm[1]}"
    data = _load(cache)
    if key in data:
        return tuple(data[key]["shape"])
    master = MucaJob(L, T, n_walkers, seed=seed, lnW=lnW, max_delta=1)
    _warm(master, *warm)
    spins, state = master.read_state()
    weights = master.lnW
    master.free()
    best, best_ms, timings = None, float("inf"), {}
    for shape in (PLAIN_SHAPES if shapes is None else shapes):
        clone = MucaJob(L, T, n_walkers, seed=seed, lnW=weights, max_delta=1)
        try:
            clone.set_launch(*shape)
        except MucaError:
            clone.free()
            continue
        clone.write_state(spins, state)
        ms = _time(clone.sweep, probe_sweeps)
        clone.free()
        timings[str(shape)] = ms
        if ms < best_ms:
            best, best_ms = shape, ms
    if best is None:
        raise ValueError(f"no valid launch shape for L={L} T={T} walkers={n_walkers}")
    data[key] = {"shape": list(best), "ms": best_ms, "probe_sweeps": probe_sweeps, "warm": list(warm),
                 "timings": timings}
    _save(cache, data)
    return best


def tune_batch(specs: Sequence[tuple], probe_sweeps: int = 100, cache: Optional[str] = None, shapes=None,
               warm: tuple = (0, 0), finalists: int = 1, repeats: int = 0) -> tuple:
    """Fastest (waves_per_walker, blocks_per_lane, blocks, packing) for a batch
    of jobs given as (L, T, n_walkers, seed) tuples (from the cache when it
    holds one).  warm as for tune_job: the batch is timed after that many
    iterations of every job.  Every valid shape is timed once; the `finalists`
    fastest are then timed `repeats` more times each, in turn, and the one with
    the least total time wins (one timing of a persistent launch varies by a
    few per cent, as much as the leading shapes differ).  ValueError if no
    candidate shape is valid."""
    sig = ",".join(f"{L}:{T!r}:{n}" for (L, T, n, _) in sorted(specs))
    rep = f"|final{finalists}x{repeats}" if finalists > 1 and repeats > 0 else ""
    key = f"batch4|{_device_name()}|{sig}|warm{warm[0]}x{warm[1]}{rep}"
    data = _load(cache)
    if key in data:
        return tuple(data[key]["shape"])
    clones = [MucaJob(L, T, n, seed=s, max_delta=1) for (L, T, n, s) in specs]
    batch = MucaBatch(clones)
    for _ in range(warm[0]):
        batch.sweep(warm[1])
        for c in clones:
            c.update_weights(c.reduce_hist())
    # every candidate starts from the same walkers (the timed sweeps move them)
    states = [c.read_state() for c in clones]
    best, best_ms, timings = None, float("inf"), {}
    if shapes is None:
        import torch
        shapes = batch_shapes(torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count)
    def timed(shape):
        batch.set_launch(*shape)
        for c, (spins, state) in zip(clones, states):
            c.write_state(spins, state)
        return _time(batch.sweep, probe_sweeps)

    valid = []
    for shape in shapes:
        try:
            ms = timed(shape)
        except MucaError:
            continue
        valid.append(shape)
        timings[str(shape)] = ms
        if ms < best_ms:
            best, best_ms = shape, ms
    final = {}
    if best is not None and finalists > 1 and repeats > 0:
        lead = sorted(valid, key=lambda s: timings[str(s)])[:finalists]
        total = {s: 0.0 for s in lead}
        for _ in range(repeats):
            for s in lead:
                total[s] += timed(s)
        best = min(lead, key=lambda s: total[s])
        best_ms = total[best] / repeats
        final = {str(s): total[s] / repeats for s in lead}
    batch.free()
    for c in clones:
        c.free()
    if best is None:
        raise ValueError(f"no valid batched launch shape for {sig}")
    data[key] = {"shape": list(best), "ms": best_ms, "probe_sweeps": probe_sweeps, "warm": list(warm),
                 "timings": timings}
    if final:
        data[key]["finalists"] = final
    _save(cache, data)
    return best


# warm-up of the benchmark tunings: (iterations, sweeps per iteration).  The
# batched workload is timed on weights past the first iterations: its later,
# steeper iterations take most of its time, and the shape fastest on the
# first ones (8 sites per lane, half the persistent blocks) is 15 % slower
# over the whole workload.
BENCH_WARM_PLAIN = (3, 2000)
BENCH_WARM_BATCH = (6, 1000)
# the batched workload's tuning: one iteration's sweeps per timing, and the
# six fastest shapes timed three more times each
BENCH_BATCH_PROBE = dict(probe_sweeps=1000, finalists=6, repeats=3)


def tune_benchmark_workloads(cache: str = CACHE) -> dict:
    """Tune the launch shapes the benchmark uses (the L=16, T=1, 1024-walker
    job and the 19-job batched workload) into cache."""
    from . import workloads

    w = workloads.workload("l16_t1_w1024")
    plain = tune_job(w["L"], w["T"], w["n_walkers"], seed=w["seed"], probe_sweeps=1000, cache=cache,
                     warm=BENCH_WARM_PLAIN)
    batch = tune_batch(workloads.batched_jobs(), cache=cache, warm=BENCH_WARM_BATCH, **BENCH_BATCH_PROBE)
    return {"l16_t1_w1024": plain, "batched": batch}


if __name__ == "__main__":
    import sys

    print(tune_benchmark_workloads(sys.argv[1] if len(sys.argv) > 1 else CACHE), flush=True)
