"""Serving loop: multicanonical jobs arriving over time, continuously batched.

Requests arrive as a Poisson process.  Each is a MUCA job (L, T, walkers,
Delta range) whose weights start tilted towards the transition field
Delta_mid(T), i.e. lnW(E) = -beta Delta_mid E, the canonical ensemble at
Delta_mid (Sec. II: one multicanonical run per temperature is reweighted to
nearby Delta).  The Delta range fixes the job's E_Delta window (the bins the
canonical distributions at the ends of the range populate, measured by two
short canonical probes, see probe_windows); the walkers are confined to it.  A
job iterates "S sweeps, merge histogram, update weights" until the merged
histogram of an iteration is flat (min/mean > threshold over its window) or it
hits the iteration cap or the run's wall budget (then it is reported as
censored).

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
    delta_range: Optional[Tuple[float, float]] = None  # None: the whole E_Delta range [0, V]


def poisson_requests(n: int, rate: float, seed: int = 0, L_range=(8, 24), T_range=(0.9, 2.0),
                     walker_choices=(64, 128, 192, 256, 320, 384, 448, 512),
                     delta_halfwidth: Optional[float] = 0.1) -> List[Request]:
    """n requests with exponential inter-arrival gaps (mean 1/rate), L uniform
    in L_range (inclusive), T uniform in T_range, walkers uniform over
    walker_choices, drawn from a seeded generator; each asks for Delta in
    Delta_mid(T) +- delta_halfwidth (None: the whole E_Delta range)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    Ls = rng.integers(L_range[0], L_range[1] + 1, size=n)
    Ts = rng.uniform(T_range[0], T_range[1], size=n)
    Ws = rng.choice(np.asarray(walker_choices), size=n)
    out = []
    for i in range(n):
        dr = None
        if delta_halfwidth is not None:
            dm = delta_mid(float(Ts[i]))
            dr = (dm - delta_halfwidth, dm + delta_halfwidth)
        out.append(Request(i, int(Ls[i]), float(Ts[i]), int(Ws[i]), int(seed * 1_000_003 + i), float(arrivals[i]), dr))
    return out


@dataclass
class ProbeConfig:
    walkers: int = 32      # walkers per probe
    relax: int = 100       # sweeps before measuring
    measure: int = 100     # sweeps measured


def _probe_margin(V: int) -> int:
    return 2 + V // 100


def probe_windows(requests: Sequence[Request], probe: ProbeConfig = ProbeConfig(),
                  retire: Optional[list] = None) -> Dict[int, Tuple[int, int]]:
    """E_Delta window of each request with a Delta range.

    Reading (the paper iterates over all of [0, V]): the window is the range
    of E_Delta that the canonical distributions at the two ends of the Delta
    range populate.  Two canonical probes per job measure it (weights
    lnW = -beta Delta_end E, probe.walkers walkers, probe.relax sweeps to
    relax, then probe.measure sweeps whose E_Delta histogram is kept): at
    Delta_lo from the fully ordered lattice (every spin +1) and at Delta_hi
    from the empty one (every spin 0), so that each starts in the phase that
    is stable at its end of the range (the low-Delta end favours occupied
    sites, the high-Delta end vacancies).  The window runs from the lowest
    E_Delta seen at Delta_hi to the highest seen at Delta_lo, widened by
    2 + V/100 bins and clipped to [0, V].  The probes of all requests run in
    one batched launch; their chains depend only on the request, so a job's
    window is the same alone and in any mix.  The probe jobs are released
    here, or appended to retire for the caller to release later."""
    reqs = [r for r in requests if r.delta_range is not None]
    if not reqs:
        return {}
    probes = []
    for r in reqs:
        V = r.L ** 3
        beta = 1.0 / r.T
        for end, (delta, fill) in enumerate(((min(r.delta_range), 1), (max(r.delta_range), 0))):
            lnW = -(beta * delta) * np.arange(V + 1, dtype=np.float64)
            job = MucaJob(r.L, r.T, probe.walkers, seed=(r.seed + ((end + 1) << 40)) & 0xFFFFFFFFFFFFFFFF,
                          lnW=lnW, max_delta=1)
            spins = np.full((probe.walkers, V), fill, dtype=np.int8)
            state = np.tile(np.array([-3 * V * fill, V * fill, V * fill, 0], dtype=np.int64), (probe.walkers, 1))
            job.write_state(spins, state)
            probes.append(job)
    batch = MucaBatch(probes) if len(probes) > 1 else None
    for sweeps in (probe.relax, probe.measure):
        if batch is not None:
            batch.sweep(sweeps)
        else:
            probes[0].sweep(sweeps)
        hists = [p.reduce_hist(reset=True) for p in probes]
    if batch is not None:
        batch.free()
    out = {}
    for k, r in enumerate(reqs):
        V = r.L ** 3
        lo_seen = np.flatnonzero(hists[2 * k + 1])
        hi_seen = np.flatnonzero(hists[2 * k])
        both = np.concatenate([lo_seen, hi_seen])
        lo, hi = int(min(lo_seen.min(), both.min())), int(max(hi_seen.max(), both.max()))
        m = _probe_margin(V)
        lo, hi = max(0, lo - m), min(V, hi + m)
        out[r.id] = (lo, hi)
    for p in probes:
        if retire is not None:
            retire.append(p)
        else:
            p.free()
    return out


@dataclass
class JobRecord:
    req: Request
    admitted: float = math.nan
    finished: float = math.nan
    iterations: int = 0
    flatness: List[float] = field(default_factory=list)
    converged: bool = False
    attempts: int = 0
    window: Tuple[int, int] = (0, 0)
    span: int = 1  # launches per iteration at the end

    @property
    def latency(self) -> float:
        return self.finished - self.req.arrival


@dataclass
class ServeConfig:
    sweeps: int = 500              # sweeps per iteration
    threshold: float = 0.5         # flatness min/mean that ends a job
    max_iterations: int = 2000     # iteration cap (job censored)
    max_walkers: int = 32768       # resident walkers
    hbm_budget: int = 16 << 30     # resident device bytes
    # batched launch shape (waves per walker, blocks per lane, persistent
    # blocks, packing) of the lanes' batches; None: the library's default
    shape: Optional[Tuple[int, int, int, int]] = None
    recursion: int = 0             # weight recursion flags (REC_ACCUMULATED | REC_EXTRAPOLATE; 0 plain)
    probe: ProbeConfig = field(default_factory=ProbeConfig)  # Delta range -> E_Delta window
    wall_budget: Optional[float] = None  # seconds; jobs unfinished by then are censored at it
    # Asynchronous lanes: resident jobs with L <= lane_bounds[0] form lane 0,
    # L <= lane_bounds[1] lane 1, ..., the rest the last lane; each lane is a
    # batch on its own stream and iterates on its own.  () = one lane: every
    # resident job advances one iteration per launch (lock-step).
    lane_bounds: Tuple[int, ...] = ()
    # Iteration length: an iteration is one launch of `sweeps` sweeps until
    # the job's histogram has visited every bin of its window; from then on
    # it spans enough launches to record about entries_per_bin entries per
    # window bin (0: always one launch).  See iteration_span.
    entries_per_bin: int = 0


# entries per window bin, above ln B, below which one launch counts as too
# short to cover a window of B bins (see iteration_span): with ln B + 3, B
# independent Poisson counts are all nonzero with probability exp(-e^-3) =
# 0.95, and the entries of a Markov chain are fewer independent ones than that
SHORT_LAUNCH_MARGIN = 3.0


def iteration_span(hist: np.ndarray, lo: int, hi: int, n_walkers: int, sweeps: int, entries_per_bin: int,
                   seen: Optional[np.ndarray] = None) -> int:
    """Launches of `sweeps` sweeps per iteration after an iteration whose
    histogram is `hist`.

    Reading (the paper fixes no iteration length): the flatness test
    min/mean > threshold is taken on one iteration's histogram, so counting
    noise alone bounds what it can show.  With n entries per bin on average
    and weights already flat, the least-visited of B bins holds about
    n - sqrt(2 n ln B) (Poisson), so at 500 sweeps of a few hundred walkers
    over thousands of bins (tens of entries per bin) the test fails about as
    often as it passes whatever the weights.  Once every bin of the window
    has been visited the weights are close enough that longer iterations
    only sharpen the test, and the iteration is stretched to about
    entries_per_bin entries per bin; before that, short iterations let the
    recursion move the weights quickly.

    A launch with fewer than ln B + SHORT_LAUNCH_MARGIN entries per bin on
    average over the B window bins leaves some bin empty often even under
    flat weights (all B Poisson counts are nonzero with probability
    exp(-B e^-m) at m entries per bin), so its iterations rarely show a
    covered window.  There the window counts as covered once the iterations
    so far (`seen`, the bins any of them visited) have covered it."""
    bins = hi - lo + 1
    covered = bool(np.all(hist[lo:hi + 1] > 0))
    if not covered and seen is not None and n_walkers * sweeps < bins * (math.log(bins) + SHORT_LAUNCH_MARGIN):
        covered = bool(np.all(seen[lo:hi + 1]))
    if entries_per_bin <= 0 or not covered:
        return 1
    return max(1, math.ceil(entries_per_bin * bins / (n_walkers * sweeps)))


class _Live:
    def __init__(self, rec: JobRecord, cfg: ServeConfig, now: float, window: Optional[Tuple[int, int]],
                 stream=None):
        r = rec.req
        self.rec = rec
        self.job = MucaJob(r.L, r.T, r.n_walkers, seed=r.seed, lnW=tilted_weights(r.L, r.T), max_delta=1)
        if cfg.recursion:
            self.job.set_recursion(cfg.recursion)
        self.V = r.L ** 3
        self.lo, self.hi = window if window is not None else (0, self.V)
        if window is not None:
            self.job.set_window(*window)
        if stream is not None:
            self.job.set_stream(stream)
        rec.window = (self.lo, self.hi)
        rec.admitted = now
        self.span = 1      # launches per iteration
        self.launches = 0  # launches of the iteration in progress
        self.seen = np.zeros(self.V + 1, dtype=bool)  # bins visited by any iteration so far

    def step_done(self, cfg: ServeConfig, now: float) -> bool:
        """After a launch: at the end of an iteration, merge its histogram
        (the device histogram accumulates over the iteration's launches) and
        finish the job or update its weights."""
        rec = self.rec
        rec.attempts += rec.req.n_walkers * self.V * cfg.sweeps
        self.launches += 1
        if self.launches < self.span:
            return False
        self.launches = 0
        h = self.job.reduce_hist(reset=True)
        f = muca_flatness(h, self.lo, self.hi)
        rec.iterations += 1
        rec.flatness.append(f)
        if f > cfg.threshold or rec.iterations >= cfg.max_iterations:
            rec.converged = f > cfg.threshold
            rec.finished = now
            return True
        self.job.update_weights(h)
        if self.span == 1:
            self.seen |= h > 0
            self.span = rec.span = iteration_span(h, self.lo, self.hi, rec.req.n_walkers, cfg.sweeps,
                                                  cfg.entries_per_bin, seen=self.seen)
        return False


def footprint(r: Request) -> int:
    return sum(muca_query_sizes(r.L, r.T, r.n_walkers, r.seed, 1).values())


def _wait_until(t0: float, t: float):
    dt = t - (time.perf_counter() - t0)
    if dt > 0:
        time.sleep(dt)


def _censor_at_budget(records: Dict[int, JobRecord], arrived: Sequence[Request], budget: float):
    """Jobs that arrived before the wall budget and have not finished are
    censored at it: latency = budget - arrival, a lower bound."""
    for r in arrived:
        rec = records.get(r.id)
        if rec is None:
            rec = records[r.id] = JobRecord(r)
        if math.isnan(rec.finished):
            rec.finished = budget
            rec.converged = False


def lane_of(L: int, bounds: Tuple[int, ...]) -> int:
    for k, b in enumerate(bounds):
        if L <= b:
            return k
    return len(bounds)


class _Lane:
    """Resident jobs of one size class, swept as one batch (or alone) on the
    lane's own stream."""

    def __init__(self, stream):
        self.stream = stream
        self.active: List[_Live] = []
        self.members: List[_Live] = []  # the jobs of the launch in flight
        self.batch = None
        self.changed = False
        self.in_flight = False

    def launch(self, cfg: ServeConfig):
        if len(self.active) == 1:
            # a lone job runs its own launch (its shape keeps neighbour
            # positions in registers and spreads few walkers over whole blocks)
            if self.batch is not None:
                self.batch.free()
                self.batch = None
            self.active[0].job.submit(cfg.sweeps)
        else:
            if self.changed or self.batch is None:
                if self.batch is not None:
                    self.batch.free()
                self.batch = MucaBatch([a.job for a in self.active])
                if cfg.shape:
                    self.batch.set_launch(*cfg.shape)
            self.batch.submit(cfg.sweeps)
        self.changed = False
        self.members = list(self.active)
        self.in_flight = True

    def done(self) -> bool:
        if len(self.members) == 1 and self.batch is None:
            return self.members[0].job.poll()
        return self.batch.poll()


def serve(requests: Sequence[Request], cfg: ServeConfig, keep_jobs: bool = False, progress=None) -> dict:
    """Continuous batching over the request stream (real time).  progress, if
    given, is called with the finished job records as jobs finish.

    Arrivals join a FIFO queue and are admitted while the resident walkers
    and device bytes fit; an admitted job's window comes from its probes and
    it joins the lane of its size.  Every lane with resident jobs and no launch
    in flight launches one iteration (S sweeps) of its jobs; a lane whose
    launch has finished merges each job's histogram, finishes the flat (or
    capped) ones and updates the others' weights, while the other lanes keep
    running.  Host resources of finished jobs are released at the end (their
    release would wait for the whole device).

    Lanes only run independently if their streams do not share a hardware
    queue: HIP maps a process's streams onto GPU_MAX_HW_QUEUES queues (4
    unless set before HIP starts), so a process serving with n lanes wants at
    least n + 1 of them (the lanes and the default stream)."""
    import torch

    t0 = time.perf_counter()
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    queue: collections.deque = collections.deque()
    arrived: List[Request] = []
    n_lanes = len(cfg.lane_bounds) + 1
    lanes = [_Lane(torch.cuda.Stream() if n_lanes > 1 else torch.cuda.current_stream()) for _ in range(n_lanes)]
    records: Dict[int, JobRecord] = {}
    kept = {}
    retired: List[MucaJob] = []
    walkers = 0
    nbytes = 0
    depth = []
    launches = 0
    attempts = 0
    host = {"probes_s": 0.0, "launch_s": 0.0, "merge_s": 0.0}
    while pending or queue or any(l.active for l in lanes):
        now = time.perf_counter() - t0
        if cfg.wall_budget is not None and now >= cfg.wall_budget:
            break
        while pending and pending[0].arrival <= now:
            r = pending.popleft()
            queue.append(r)
            arrived.append(r)
        admit = []
        resident = any(l.active for l in lanes)
        while queue:
            r = queue[0]
            fb = footprint(r)
            if (resident or admit) and (walkers + r.n_walkers > cfg.max_walkers or nbytes + fb > cfg.hbm_budget):
                break
            queue.popleft()
            admit.append(r)
            walkers += r.n_walkers
            nbytes += fb
        if admit:
            # the admitted jobs' windows: their probes in one batched launch
            th = time.perf_counter()
            windows = probe_windows(admit, cfg.probe, retired)
            host["probes_s"] += time.perf_counter() - th
            for r in admit:
                rec = JobRecord(r)
                records[r.id] = rec
                lane = lanes[lane_of(r.L, cfg.lane_bounds)]
                lane.active.append(_Live(rec, cfg, time.perf_counter() - t0, windows.get(r.id),
                                         lane.stream if n_lanes > 1 else None))
                lane.changed = True
        depth.append(len(queue))
        th = time.perf_counter()
        for lane in lanes:
            if lane.active and not lane.in_flight:
                lane.launch(cfg)
                launches += 1
                attempts += sum(a.rec.req.n_walkers * a.V for a in lane.members) * cfg.sweeps
        host["launch_s"] += time.perf_counter() - th
        if not any(l.in_flight for l in lanes):
            if pending:
                _wait_until(t0, pending[0].arrival if cfg.wall_budget is None
                            else min(pending[0].arrival, cfg.wall_budget))
            continue
        progressed = False
        for lane in lanes:
            if not (lane.in_flight and lane.done()):
                continue
            lane.in_flight = False
            progressed = True
            th = time.perf_counter()
            now = th - t0
            done = [a for a in lane.members if a.step_done(cfg, now)]
            host["merge_s"] += time.perf_counter() - th
            if not done:
                continue
            if progress is not None:
                progress([a.rec for a in done])
            for a in done:
                walkers -= a.rec.req.n_walkers
                nbytes -= footprint(a.rec.req)
                if keep_jobs:
                    kept[a.rec.req.id] = a.job
                else:
                    retired.append(a.job)
            lane.active = [a for a in lane.active if a not in done]
            lane.changed = True
        if not progressed:
            time.sleep(2e-4)
    for lane in lanes:
        if lane.batch is not None:
            lane.batch.free()
    torch.cuda.synchronize()
    if cfg.wall_budget is not None and (pending or queue or any(l.active for l in lanes)):
        _censor_at_budget(records, arrived, cfg.wall_budget)
        for lane in lanes:
            for a in lane.active:
                if keep_jobs:
                    kept[a.rec.req.id] = a.job
                else:
                    retired.append(a.job)
    makespan = time.perf_counter() - t0
    for j in retired:
        j.free()
    out = _summary(records, makespan, attempts, launches, depth, kept)
    out["not_arrived"] = len(pending)
    out["lanes"] = n_lanes
    # host time of the loop: probes of admitted jobs, launches (including
    # rebuilding a lane's batch), merges and weight updates
    out["host_s"] = dict(host)
    return out


def serve_plain(requests: Sequence[Request], cfg: ServeConfig, keep_jobs: bool = False) -> dict:
    """Baseline: the same requests, one job at a time in arrival order, each
    with its own probes and plain launches."""
    import torch

    t0 = time.perf_counter()
    records: Dict[int, JobRecord] = {}
    kept = {}
    attempts = 0
    launches = 0
    order = sorted(requests, key=lambda r: r.arrival)
    arrived: List[Request] = []
    out_of_time = False
    for r in order:
        if cfg.wall_budget is not None and max(r.arrival, time.perf_counter() - t0) >= cfg.wall_budget:
            out_of_time = True
            break
        _wait_until(t0, r.arrival)
        arrived.append(r)
        rec = JobRecord(r)
        records[r.id] = rec
        live = _Live(rec, cfg, time.perf_counter() - t0, probe_windows([r], cfg.probe).get(r.id))
        while True:
            if cfg.wall_budget is not None and time.perf_counter() - t0 >= cfg.wall_budget:
                out_of_time = True
                break
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
        if out_of_time:
            break
    not_arrived = 0
    if out_of_time:
        late = [r for r in order if r.arrival < cfg.wall_budget]
        _censor_at_budget(records, late, cfg.wall_budget)
        not_arrived = len(order) - len(late)
    makespan = time.perf_counter() - t0
    out = _summary(records, makespan, attempts, launches, [0], kept)
    out["not_arrived"] = not_arrived
    return out


def _summary(records, makespan, attempts, launches, depth, kept) -> dict:
    lat = np.array([r.latency for r in records.values()])
    conv = [r for r in records.values() if r.converged]
    out = {
        "jobs": len(records),
        "converged": len(conv),
        "censored": len(records) - len(conv),
        "makespan_s": makespan,
        "jobs_per_s": len(records) / makespan if makespan > 0 else 0.0,
        "converged_per_s": len(conv) / makespan if makespan > 0 else 0.0,
        "attempts": attempts,
        "attempts_per_s": attempts / makespan if makespan > 0 else 0.0,
        "launches": launches,
        "latency_p50_s": float(np.percentile(lat, 50)) if len(lat) else math.nan,
        "latency_p99_s": float(np.percentile(lat, 99)) if len(lat) else math.nan,
        # the same over the jobs that reached a flat histogram (censored jobs left out)
        "latency_converged_p50_s": float(np.percentile([r.latency for r in conv], 50)) if conv else math.nan,
        "latency_converged_p99_s": float(np.percentile([r.latency for r in conv], 99)) if conv else math.nan,
        "iterations_p50": float(np.percentile([r.iterations for r in records.values()], 50)) if records else 0,
        "long_iteration_jobs": sum(1 for r in records.values() if r.span > 1),
        "queue_depth_max": int(max(depth)) if depth else 0,
        "queue_depth_mean": float(np.mean(depth)) if depth else 0.0,
        "records": records,
    }
    if kept:
        out["jobs_kept"] = kept
    return out
