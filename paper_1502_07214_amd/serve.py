"""Serving loop: multicanonical jobs arriving over time, continuously batched.

Requests arrive as a Poisson process.  Each is a MUCA job (L, T, walkers)
whose weights start tilted towards the transition field Delta_mid(T), i.e.
lnW(E) = -beta Delta_mid E, the canonical ensemble at Delta_mid (Sec. II: one
multicanonical run per temperature is reweighted to nearby Delta).  A job
iterates "S sweeps, merge histogram, update weights" until the merged
histogram of an iteration is flat (min/mean > threshold over its E_Delta
window) or it hits the iteration cap (then it is reported as censored).

Continuous batching: jobs are admitted from a FIFO queue while the resident
walker count and device-memory footprint allow; every iteration of the loop is
one persistent batched launch (MucaBatch) over all resident jobs, whatever
their size (a job resident alone runs its own launch instead); finished jobs
leave and queued ones join at the next launch, so their work overlaps on the
device.  Walker state stays resident in HBM for a
job's whole life.  The per-job chain does not depend on the mix: a job served
among others gives bit-identical results to the same job run alone.

Delta_mid(T) interpolates piecewise-linearly through the transition fields
the paper reports: Delta*(T=0.9) = 2.964, Delta*(T=1.0) = 2.944 (Sec. III,
first-order regime), Delta_t = 2.8446 at T_t = 1.4182 (tricritical estimate)
and Delta_c(T=2.0) = 2.523 (second-order regime).
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .muca import MucaBatch, MucaJob, muca_flatness, muca_query_sizes

TRANSITION = ((0.9, 2.964), (1.0, 2.944), (1.4182, 2.8446), (2.0, 2.523))


def delta_mid(T: float) -> float:
    Ts = [t for t, _ in TRANSITION]
    Ds = [d for _, d in TRANSITION]
    return float(np.interp(T, Ts, Ds))


def tilted_weights(L: int, T: float) -> np.ndarray:
    V = L ** 3
    return -(1.0 / T) * delta_mid(T) * np.arange(V + 1, dtype=np.float64)


@dataclass
class Request:
    id: int
    L: int
    T: float
    n_walkers: int
    seed: int
    arrival: float  # seconds after the start of the run


def poisson_requests(n: int, rate: float, seed: int = 0, L_range=(8, 24), T_range=(0.9, 2.0),
                     walker_choices=(64, 128, 192, 256, 320, 384, 448, 512)) -> List[Request]:
    """n requests with exponential inter-arrival gaps (mean 1/rate), L uniform
    in L_range (inclusive), T uniform in T_range, walkers uniform over
    walker_choices; drawn from a seeded generator."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    Ls = rng.integers(L_range[0], L_range[1] + 1, size=n)
    Ts = rng.uniform(T_range[0], T_range[1], size=n)
    Ws = rng.choice(np.asarray(walker_choices), size=n)
    return [Request(i, int(Ls[i]), float(Ts[i]), int(Ws[i]), int(seed * 1_000_003 + i), float(arrivals[i]))
            for i in range(n)]


@dataclass
class JobRecord:
    req: Request
    admitted: float = math.nan
    finished: float = math.nan
    iterations: int = 0
    flatness: List[float] = field(default_factory=list)
    converged: bool = False
    attempts: int = 0

    @property
    def latency(self) -> float:
        return self.finished - self.req.arrival


@dataclass
class ServeConfig:
    sweeps: int = 500              # sweeps per iteration
    threshold: float = 0.5         # flatness min/mean that ends a job
    max_iterations: int = 2000     # iteration cap (job censored)
    window: Tuple[float, float] = (0.0, 1.0)  # flatness window as fractions of V
    max_walkers: int = 32768       # resident walkers
    hbm_budget: int = 16 << 30     # resident device bytes
    shape: Optional[Tuple[int, int]] = None  # batched launch shape (None: library default)
    recursion: int = 0             # weight recursion flags (REC_ACCUMULATED | REC_EXTRAPOLATE; 0 plain)


class _Live:
    def __init__(self, rec: JobRecord, cfg: ServeConfig, now: float):
        r = rec.req
        self.rec = rec
        self.job = MucaJob(r.L, r.T, r.n_walkers, seed=r.seed, lnW=tilted_weights(r.L, r.T), max_delta=1)
        if cfg.recursion:
            self.job.set_recursion(cfg.recursion)
        self.V = r.L ** 3
        self.lo = int(round(cfg.window[0] * self.V))
        self.hi = int(round(cfg.window[1] * self.V))
        rec.admitted = now

    def step_done(self, cfg: ServeConfig, now: float) -> bool:
        """Merge the iteration's histogram; finish or update the weights."""
        h = self.job.reduce_hist(reset=True)
        f = muca_flatness(h, self.lo, self.hi)
        rec = self.rec
        rec.iterations += 1
        rec.flatness.append(f)
        rec.attempts += rec.req.n_walkers * self.V * cfg.sweeps
        if f > cfg.threshold or rec.iterations >= cfg.max_iterations:
            rec.converged = f > cfg.threshold
            rec.finished = now
            return True
        self.job.update_weights(h)
        return False


def footprint(r: Request) -> int:
    return sum(muca_query_sizes(r.L, r.T, r.n_walkers, r.seed, 1).values())


def _wait_until(t0: float, t: float):
    dt = t - (time.perf_counter() - t0)
    if dt > 0:
        time.sleep(dt)


def serve(requests: Sequence[Request], cfg: ServeConfig, keep_jobs: bool = False, progress=None) -> dict:
    """Continuous batching over the request stream (real time).  progress, if
    given, is called with the finished job records as jobs finish."""
    import torch

    t0 = time.perf_counter()
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    queue: collections.deque = collections.deque()
    active: List[_Live] = []
    records: Dict[int, JobRecord] = {}
    kept = {}
    batch = None
    walkers = 0
    nbytes = 0
    depth = []
    launches = 0
    attempts = 0
    while pending or queue or active:
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            queue.append(pending.popleft())
        changed = False
        while queue:
            r = queue[0]
            fb = footprint(r)
            if active and (walkers + r.n_walkers > cfg.max_walkers or nbytes + fb > cfg.hbm_budget):
                break
            queue.popleft()
            rec = JobRecord(r)
            records[r.id] = rec
            active.append(_Live(rec, cfg, time.perf_counter() - t0))
            walkers += r.n_walkers
            nbytes += fb
            changed = True
        depth.append(len(queue))
        if not active:
            _wait_until(t0, pending[0].arrival)
            continue
        if len(active) == 1:
            # a lone job runs its own launch (its shape keeps neighbour
            # positions in registers and spreads few walkers over whole blocks)
            if batch is not None:
                batch.free()
                batch = None
            active[0].job.sweep(cfg.sweeps)
        else:
            if changed or batch is None:
                if batch is not None:
                    batch.free()
                batch = MucaBatch([a.job for a in active])
                if cfg.shape:
                    batch.set_launch(*cfg.shape)
            batch.sweep(cfg.sweeps)
        launches += 1
        attempts += sum(a.rec.req.n_walkers * a.V for a in active) * cfg.sweeps
        torch.cuda.current_stream().synchronize()
        now = time.perf_counter() - t0
        done = [a for a in active if a.step_done(cfg, now)]
        if done:
            if batch is not None:
                batch.free()
                batch = None
            if progress is not None:
                progress([a.rec for a in done])
            for a in done:
                walkers -= a.rec.req.n_walkers
                nbytes -= footprint(a.rec.req)
                if keep_jobs:
                    kept[a.rec.req.id] = a.job
                else:
                    a.job.free()
            active = [a for a in active if a not in done]
    if batch is not None:
        batch.free()
    makespan = time.perf_counter() - t0
    return _summary(records, makespan, attempts, launches, depth, kept)


def serve_plain(requests: Sequence[Request], cfg: ServeConfig, keep_jobs: bool = False) -> dict:
    """Baseline: the same requests, one job at a time in arrival order, each
    with its own plain launches."""
    import torch

    t0 = time.perf_counter()
    records: Dict[int, JobRecord] = {}
    kept = {}
    attempts = 0
    launches = 0
    for r in sorted(requests, key=lambda r: r.arrival):
        _wait_until(t0, r.arrival)
        rec = JobRecord(r)
        records[r.id] = rec
        live = _Live(rec, cfg, time.perf_counter() - t0)
        while True:
            live.job.sweep(cfg.sweeps)
            launches += 1
            attempts += r.n_walkers * live.V * cfg.sweeps
            torch.cuda.current_stream().synchronize()
            if live.step_done(cfg, time.perf_counter() - t0):
                break
        if keep_jobs:
            kept[r.id] = live.job
        else:
            live.job.free()
    makespan = time.perf_counter() - t0
    return _summary(records, makespan, attempts, launches, [0], kept)


def _summary(records, makespan, attempts, launches, depth, kept) -> dict:
    lat = np.array([r.latency for r in records.values()])
    conv = [r for r in records.values() if r.converged]
    out = {
        "jobs": len(records),
        "converged": len(conv),
        "censored": len(records) - len(conv),
        "makespan_s": makespan,
        "jobs_per_s": len(records) / makespan if makespan > 0 else 0.0,
        "attempts": attempts,
        "attempts_per_s": attempts / makespan if makespan > 0 else 0.0,
        "launches": launches,
        "latency_p50_s": float(np.percentile(lat, 50)) if len(lat) else math.nan,
        "latency_p99_s": float(np.percentile(lat, 99)) if len(lat) else math.nan,
        # the same over the jobs that reached a flat histogram (censored jobs left out)
        "latency_converged_p50_s": float(np.percentile([r.latency for r in conv], 50)) if conv else math.nan,
        "latency_converged_p99_s": float(np.percentile([r.latency for r in conv], 99)) if conv else math.nan,
        "iterations_p50": float(np.percentile([r.iterations for r in records.values()], 50)) if records else 0,
        "queue_depth_max": int(max(depth)) if depth else 0,
        "queue_depth_mean": float(np.mean(depth)) if depth else 0.0,
        "records": records,
    }
    if kept:
        out["jobs_kept"] = kept
    return out
