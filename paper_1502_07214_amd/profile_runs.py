"""Fixed workloads for rocprofv3 runs.

    python -m paper_1502_07214_amd.profile_runs copy    # plain device copy of 1 GiB, 3 times
    python -m paper_1502_07214_amd.profile_runs sweep   # the benchmark's sweep launches (L=12, 256 walkers)
    python -m paper_1502_07214_amd.profile_runs saturation  # L=8, 65 536 walkers, 10 + 100 sweeps
    python -m paper_1502_07214_amd.profile_runs satgrid     # L=8, 12, 16 x 65 536 .. 262 144 walkers, 10 + 100 sweeps
    python -m paper_1502_07214_amd.profile_runs served      # the served stream in asynchronous lanes, 40 s
    python -m paper_1502_07214_amd.profile_runs batched     # 19 mixed jobs: 10 batched launches of 1000 sweeps
    python -m paper_1502_07214_amd.profile_runs c3          # L=16, T=1, 1024 walkers: 3 iterations of 2*10^4 sweeps
    python -m paper_1502_07214_amd.profile_runs bigL L W P  # L^3, W walkers, packing P (0, 1, -1 auto): 3 x 200 sweeps

`copy` calibrates the FETCH_SIZE / WRITE_SIZE counters: each copy moves exactly
2^30 bytes in and 2^30 bytes out of HBM, so counter / 2^30 is the factor that
turns the counters of other kernels into bytes.  `sweep` runs three
iterations of the benchmark job (10^4 sweeps of 256 walkers at L = 12, T = 2,
each followed by the histogram merge and weight update).  `saturation` and
`batched` are the saturation job and the batched workload of the benchmark
(its batched mode only).
"""
from __future__ import annotations

import sys


def copy(nbytes: int = 1 << 30, reps: int = 3):
    import torch

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {nbytes} bytes x {reps}", flush=True)


def sweep(iterations: int = 3):
    import torch

    from . import MucaJob, workloads

    w = workloads.workload("l12_t2_w256")
    job = MucaJob(w["L"], w["T"], w["n_walkers"], seed=w["seed"], max_delta=1)
    for it in range(iterations):
        job.sweep(w["sweeps"])
        job.update_weights(job.reduce_hist())
        print(f"iteration {it} done", flush=True)
    torch.cuda.synchronize()
    job.free()


def saturation():
    import torch

    from . import MucaJob, workloads

    s = workloads.SATURATION
    job = MucaJob(s["L"], s["T"], s["n_walkers"], seed=s["seed"], max_delta=1)
    job.sweep(10)
    job.sweep(s["sweeps"])
    torch.cuda.synchronize()
    print(f"saturation: {s['n_walkers']} walkers at L={s['L']}, 10 + {s['sweeps']} sweeps", flush=True)
    job.free()


def saturation_grid():
    """The saturation grid: L = 8, 12, 16 with 65 536, 131 072 and 262 144
    walkers (flat weights, T = 2), each 10 + 100 sweeps in the library's
    launch shape, in the grid's order."""
    import torch

    from . import MucaJob, workloads

    s = workloads.SATURATION
    for (L, n) in workloads.SATURATION_GRID:
        job = MucaJob(L, s["T"], n, seed=s["seed"], max_delta=1)
        job.sweep(10)
        job.sweep(s["sweeps"])
        torch.cuda.synchronize()
        print(f"saturation grid: L={L} walkers={n} launch {job.get_launch()}, 10 + {s['sweeps']} sweeps", flush=True)
        job.free()


def served():
    """The served stream as the benchmark serves it in asynchronous lanes
    (200 jobs, L 8..24, 40 s wall budget), once."""
    from . import REC_ACCUMULATED, REC_EXTRAPOLATE, workloads
    from .serve import ServeConfig, poisson_requests, serve

    sp = workloads.SERVED
    reqs = poisson_requests(sp["n_jobs"], sp["rate"], sp["seed"], sp["L_range"], sp["T_range"], sp["walker_choices"],
                            delta_halfwidth=sp["delta_halfwidth"])
    cfg = ServeConfig(sweeps=sp["sweeps"], threshold=sp["threshold"], max_iterations=sp["max_iterations"],
                      wall_budget=sp["wall_budget"], recursion=REC_ACCUMULATED | REC_EXTRAPOLATE,
                      lane_bounds=tuple(sp["lane_bounds"]), entries_per_bin=sp["entries_per_bin"])
    r = serve(reqs, cfg)
    print(f"served: {r['converged']} of {r['jobs']} flat, p50 {r['latency_p50_s']:.2f} s, "
          f"{r['attempts_per_s']:.3e} attempts/s, {r['launches']} launches", flush=True)


def batched(tuned: bool = False):
    """The benchmark's batched workload, lock-step, in the default batch shape
    or (tuned) in the one the benchmark tunes for it (from the committed
    tuning cache)."""
    import torch

    from . import MucaBatch, MucaJob, autotune, workloads

    specs = workloads.batched_jobs()
    jobs = [MucaJob(L, T, n, seed=sd, max_delta=1) for (L, T, n, sd) in specs]
    batch = MucaBatch(jobs)
    if tuned:
        shape = autotune.tune_batch(specs, cache=autotune.CACHE, warm=autotune.BENCH_WARM_BATCH,
                                    **autotune.BENCH_BATCH_PROBE)
        batch.set_launch(*shape)
        print(f"batched launch {shape}", flush=True)
    for it in range(workloads.BATCHED["iterations"]):
        batch.sweep(workloads.BATCHED["sweeps"])
        for j in jobs:
            j.update_weights(j.reduce_hist())
        print(f"batched iteration {it} done", flush=True)
    torch.cuda.synchronize()
    batch.free()
    for j in jobs:
        j.free()


def c3(iterations: int = 3):
    """The L=16, T=1, 1024-walker job in the launch shape the benchmark
    tunes for it (from the committed tuning cache)."""
    import torch

    from . import MucaJob, autotune, workloads

    w = workloads.workload("l16_t1_w1024")
    shape = autotune.tune_job(w["L"], w["T"], w["n_walkers"], seed=w["seed"], probe_sweeps=1000,
                              cache=autotune.CACHE, warm=autotune.BENCH_WARM_PLAIN)
    job = MucaJob(w["L"], w["T"], w["n_walkers"], seed=w["seed"], max_delta=1)
    job.set_launch(*shape)
    print(f"c3 launch {job.get_launch()}", flush=True)
    for it in range(iterations):
        job.sweep(w["sweeps"])
        job.update_weights(job.reduce_hist())
        print(f"iteration {it} done", flush=True)
    torch.cuda.synchronize()
    job.free()


def bigL(L: int, walkers: int, packing: int, iterations: int = 3, sweeps: int = 200):
    """A large lattice with many walkers (one wave per walker, thresholds
    through the caches), lattices packed or not: 3 iterations of 200 sweeps
    from a flat start."""
    import torch

    from . import MucaJob

    job = MucaJob(L, 2.0, walkers, seed=7, max_delta=1)
    job.set_launch(1, 1, 0, packing)
    print(f"bigL L={L} walkers={walkers} launch {job.get_launch()}", flush=True)
    for it in range(iterations):
        job.sweep(sweeps)
        job.update_weights(job.reduce_hist())
        print(f"iteration {it} done", flush=True)
    torch.cuda.synchronize()
    job.free()


if __name__ == "__main__":
    if sys.argv[1] == "bigL":
        bigL(int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4]))
    else:
        {"copy": copy, "sweep": sweep, "saturation": saturation, "satgrid": saturation_grid, "batched": batched,
         "batched_tuned": lambda: batched(tuned=True), "c3": c3, "served": served}[sys.argv[1]]()
