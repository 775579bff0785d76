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
