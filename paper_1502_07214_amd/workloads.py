"""Seeded synthetic workloads of the paper's kind, shared by tests and the benchmark.

Holds only sizes, seeds and schedules: no arithmetic of the method.  All random
draws of the method itself (initial lattices, proposals, uniforms) come from the
counter-based Philox streams that each implementation computes on its own.

The shapes follow the paper: periodic simple cubic lattices with L in 8..28
(Sec. II), temperatures T in {0.9, 1.0} (first-order regime), 2.0 (second
order) and the tricritical estimate 1.4182 (Sec. I), a parallel width of dozens
to thousands of independent walkers, and a Delta grid across the transition
(Delta_c(T=2) about 2.52, Sec. III).
"""
from __future__ import annotations

import numpy as np

# name: (L, T, n_walkers, seed, iterations, sweeps per iteration, production sweeps, n_delta)
PLAIN = {
    # L=4, T=2.0, 16 walkers, flat start, 10 iterations x 2000 sweeps
    "l4_t2_w16": dict(L=4, T=2.0, n_walkers=16, seed=0, iterations=10, sweeps=2000,
                      production=2000, deltas=(0.0, 3.0, 200)),
    # L=12, T=2.0 (second-order regime), 256 walkers, 30 iterations x 10^4 sweeps,
    # reweighted to 200 Delta values in [0, 3]
    "l12_t2_w256": dict(L=12, T=2.0, n_walkers=256, seed=0, iterations=30, sweeps=10000,
                        production=10000, deltas=(0.0, 3.0, 200)),
    # L=16, T=1.0 (first-order regime), 1024 walkers, 60 iterations x 2*10^4 sweeps
    "l16_t1_w1024": dict(L=16, T=1.0, n_walkers=1024, seed=0, iterations=60, sweeps=20000,
                         production=20000, deltas=(2.5, 3.2, 200)),
}

# Truncated schedules of the same jobs: same walkers and initial state, fewer
# sweeps, so that the oracle finishes in seconds.
TRUNCATED = {
    "l12_t2_w256": dict(iterations=2, sweeps=1000, production=500),
    "l16_t1_w1024": dict(iterations=2, sweeps=100, production=100),
}


def delta_grid(spec) -> np.ndarray:
    lo, hi, n = spec
    return np.linspace(lo, hi, int(n))


def workload(name: str, truncated: bool = False) -> dict:
    w = dict(PLAIN[name])
    if truncated:
        w.update(TRUNCATED[name])
    w["name"] = name + ("_truncated" if truncated else "")
    w["V"] = w["L"] ** 3
    w["attempts"] = w["n_walkers"] * w["V"] * (w["iterations"] * w["sweeps"] + w["production"])
    return w


# Batched: 4096 walkers in 64 groups of 64; each group's (L, T) drawn uniformly
# from {8,10,12,16,20} x {0.9,1.0,1.4182,2.0} by a seeded generator; groups
# with equal (L, T) form one job (one histogram, one weight function);
# 10 iterations x 1000 sweeps from flat weights.
BATCHED = dict(groups=64, group_walkers=64, Ls=(8, 10, 12, 16, 20), Ts=(0.9, 1.0, 1.4182, 2.0), seed=0,
               iterations=10, sweeps=1000)


def batched_jobs(spec=BATCHED) -> list:
    """[(L, T, n_walkers, seed)] of the batched workload, one entry per job."""
    rng = np.random.default_rng(spec["seed"])
    combos = [(L, T) for L in spec["Ls"] for T in spec["Ts"]]
    picks = rng.integers(0, len(combos), size=spec["groups"])
    counts = {}
    for p in picks:
        counts[combos[p]] = counts.get(combos[p], 0) + spec["group_walkers"]
    # one Philox key per (L, T): 10^4 T < 10^5 for every temperature here, so the map is one-to-one
    return [(L, T, n, 100_000 * L + int(round(T * 1e4))) for (L, T), n in sorted(counts.items())]


# Served: Poisson arrivals (mean 20 jobs/s, seed 0) of 200 MUCA jobs, L
# uniform in 8..24, T uniform in [0.9, 2.0], 64..512 walkers (multiples of
# 64), each asking for Delta in Delta_mid(T) +- 0.1 (its E_Delta window comes
# from two canonical probes), weights tilted to Delta_mid(T), 500 sweeps per
# iteration until the histogram over the window is flat (min/mean > 0.5), cap
# 2000 iterations; the run stops at a wall budget and the jobs unfinished by
# then are censored at it.  Lanes: L <= 12, <= 16, <= 20, larger.
SERVED = dict(n_jobs=200, rate=20.0, seed=0, L_range=(8, 24), T_range=(0.9, 2.0),
              walker_choices=(64, 128, 192, 256, 320, 384, 448, 512), delta_halfwidth=0.1, sweeps=500,
              threshold=0.5, max_iterations=2000, wall_budget=40.0, lane_bounds=(12, 16, 20),
              entries_per_bin=200)

# Lanes of the batched workload when its jobs iterate asynchronously (L <= 8,
# 10, 12, 16, larger).
BATCHED_LANES = (8, 10, 12, 16)

# Saturation: enough walkers to fill every SIMD several times over (roofline run).
SATURATION = dict(L=8, T=2.0, n_walkers=65536, seed=0, sweeps=100)
# The saturation runs over lattice sizes and walker counts: 1024 SIMDs x 64
# lanes x 1, 2, 4 waves of walkers at L = 8, 12, 16 (flat weights, T = 2).
SATURATION_GRID = tuple((L, n) for L in (8, 12, 16) for n in (65536, 131072, 262144))

# Time to a flat histogram (min/mean > 0.5 over [0, V]) for single jobs, with
# the plain recursion and with the accumulated + extrapolating one, from a flat
# start and from the start tilted towards the transition field.  With the plain
# recursion from a flat start, L = 12 needs at least
# (3 beta V + ln 2) / ln(walkers x sweeps) ~ 200 iterations at these sizes.
CONVERGENCE = (
    dict(L=8, T=2.0, n_walkers=256, seed=0, sweeps=500, threshold=0.5, max_iterations=400),
    dict(L=12, T=2.0, n_walkers=256, seed=0, sweeps=2000, threshold=0.5, max_iterations=300),
)
