#!/usr/bin/env python3
"""Benchmark: spin-flip attempts per second of plain parallel multicanonical
sampling of the 3D Blume-Capel model on one MI355X.

Workload (one "step"): L=12 (V=1728), T=2.0, 256 walkers, flat start, 30
iterations of 10^4 sweeps each (sweep, merge histograms, update weights), then
10^4 production sweeps recording per-bin sums and reweighting to 200 Delta
values in [0, 3].  Every step re-initialises the job from the same seed.
attempts per step = 256 * 1728 * (30 * 10^4 + 10^4) = 1.371e11.

Prints one JSON line.  The sweep kernel's average launch duration is measured
with HIP events on the job's stream over the timed region; its roofline uses
the algorithmic VALU work per attempt (see ALGO_SLOTS_PER_ATTEMPT).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/sec on 1 GPU (plain vs batched/served) + p99 time-to-flat-histogram"
WORKLOAD = "l12_t2_w256"

# Algorithmic VALU issue slots per attempt (one site visit), counted from what
# the method must compute: a quarter of a Philox4x32-10 block (10 rounds of two
# 32x32->64 products at 4 slots per 32-bit multiply half and 4 XORs) = 50; the
# six-neighbour sum 5; proposal 4; dS, dE_J, dE_Delta 5; u31 to double 3; the
# threshold product and compare (FP64, 2 slots each) 4; E_J/E_Delta/M updates 3;
# the spin write-back select 1.
ALGO_SLOTS_PER_ATTEMPT = 75
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz full-rate VALU lane slots.
PEAK_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default=None, help="wpw,bpl,lds_tables (default: library's choice)")
    return ap.parse_args()


def run_step(w, deltas, events=None, launch=None):
    import torch

    from paper_1502_07214_amd import MucaJob

    job = MucaJob(w["L"], w["T"], w["n_walkers"], seed=w["seed"], max_delta=len(deltas))
    if launch:
        job.set_launch(*launch)
    flat = 0.0
    for it in range(w["iterations"]):
        if events is not None:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            job.sweep(w["sweeps"])
            e1.record()
            events.append((e0, e1))
        else:
            job.sweep(w["sweeps"])
        h = job.reduce_hist(reset=True)
        flat = job.update_weights(h)
    job.sweep(w["production"], record=True)
    job.reduce_hist(reset=True)
    obs = job.reweight(deltas)
    shape = job.get_launch()
    job.free()
    return flat, obs, shape


def cpu_baseline(w, deltas):
    """The oracle as it stands, on the truncated schedule of the same job."""
    import oracle
    from paper_1502_07214_amd import workloads

    t = workloads.workload(w["name"].replace("_truncated", ""), truncated=True)
    t0 = time.perf_counter()
    o = oracle.OracleJob(t["L"], t["T"], t["n_walkers"], t["seed"])
    for it in range(t["iterations"]):
        o.sweep(t["sweeps"])
        o.update_weights(o.take_hist())
    o.sweep(t["production"], record=True)
    o.take_hist()
    o.reweight(deltas)
    dt = time.perf_counter() - t0
    return {"value": t["attempts"] / dt, "unit": "attempts/s", "cores": o.threads_used, "kind": "oracle",
            "sample": f"{t['name']}: all {t['n_walkers']} walkers, {t['iterations']} x {t['sweeps']} sweeps + "
                      f"{t['production']} production sweeps + reweight to {len(deltas)} Delta "
                      f"({t['attempts']:.3e} attempts, {dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not part of this build",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1502_07214_amd import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = workloads.workload(args.workload)
    deltas = workloads.delta_grid(w["deltas"])
    launch = tuple(int(x) for x in args.launch.split(",")) if args.launch else None
    print(f"[bench] workload {w['name']}: {w['attempts']:.4e} attempts/step, warmup {args.warmup}, "
          f"steps {args.steps}", file=sys.stderr, flush=True)

    for k in range(args.warmup):
        run_step(w, deltas, launch=launch)
        print(f"[bench] warmup step {k} done", file=sys.stderr, flush=True)

    events = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flat, obs, shape = 0.0, None, None
    for k in range(args.steps):
        flat, obs, shape = run_step(w, deltas, events=events, launch=launch)
        print(f"[bench] step {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    attempts_per_launch = w["n_walkers"] * w["V"] * w["sweeps"]
    kernel_rate = attempts_per_launch / (launch_ms * 1e-3)
    achieved = attempts_per_launch * ALGO_SLOTS_PER_ATTEMPT / (launch_ms * 1e-3)
    value = args.steps * w["attempts"] / elapsed

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32+f64",
        "data": "synthetic (seeded Philox initial lattices; the Monte Carlo chain is the workload)",
        "config": {"workload": w["name"], "L": w["L"], "T": w["T"], "walkers": w["n_walkers"],
                   "iterations": w["iterations"], "sweeps_per_iteration": w["sweeps"],
                   "production_sweeps": w["production"], "n_delta": len(deltas), "launch": shape},
        "kernel_attempts_per_s": kernel_rate,
        "sweep_launch_ms": launch_ms,
        "final_flatness": flat,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS_PER_S / 1e12,
                     "unit": "Tslot/s", "frac": achieved / PEAK_SLOTS_PER_S, "traffic": None,
                     "kernel": "muca_sweep_kernel", "slots_per_attempt": ALGO_SLOTS_PER_ATTEMPT},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, deltas)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
