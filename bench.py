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
import dataclasses
import json
import os
import sys
import time

# The served leg runs its lanes on separate HIP streams.  HIP maps a process's
# streams onto GPU_MAX_HW_QUEUES hardware queues (4 unless set), and streams
# that share a queue run in submission order: a histogram read on one lane
# then waits for another lane's kernel (measured: the loop spent 27 of 40 s
# blocked in such reads, with 40 % fewer launches).  Eight queues give each
# lane and the default stream one of their own.  HIP reads the variable when
# it starts, so it is set before torch is imported; a larger value is kept.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/sec on 1 GPU (plain vs batched/served) + p99 time-to-flat-histogram"
WORKLOAD = "l12_t2_w256"

# Algorithmic VALU issue per attempt (one site visit), in full-rate lane slots
# (a full-rate wave64 VALU instruction = 64 lane slots): the 45-55 slot-
# equivalents counted for the method's work (a quarter of a Philox4x32-10
# block, six neighbour reads and their sum, class and index arithmetic, one
# u32 -> f64 convert, one FP64 product and compare, a 2-bit write, three
# conditional integer updates, 1/V of a histogram atomic), taken at the
# midpoint.  The itemised count with the instruction rates measured on MI355X
# (v_xor_b32, v_mul_f64, v_cvt_f64_u32 full rate, v_mad_u64_u32 1.5x) is 32.5:
#   a quarter of a Philox4x32-10 block: 5 32x32->64 products (7.5) and 5
#   three-input XORs (5) = 12.5; six-neighbour sum 3; proposal 3; dS, dE_J,
#   dE_Delta 4; u31 to double 2; B' index 1; FP64 threshold product and compare
#   2; E_J/E_Delta/M updates 3; spin write-back select 1; class/validity 1.
ALGO_SLOTS_PER_ATTEMPT = 50.0
ITEMISED_SLOTS_PER_ATTEMPT = 32.5
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz full-rate VALU lane slots.
PEAK_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
# HBM bytes per 10^4-sweep launch of muca_sweep_kernel<4,1,false,true,2> on this
# workload, averaged over the 30 iteration launches of one step of this script:
# FETCH_SIZE + WRITE_SIZE from rocprofv3, each scaled by the same counter's
# reading on a plain 1 GiB copy (profiles/sweep_kernel_l12_t2_w256_pmc.txt).
TRAFFIC_KERNEL = "muca_sweep_kernel<4, 1, false, true, 2, false>"
TRAFFIC_BYTES_PER_LAUNCH = 2316231
# weight recursions of the convergence legs (flags of muca_set_recursion)
REC_EXTRAPOLATE, REC_ACC_EXT = 2, 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1, help="number of GPUs (only 1 is supported)")
    ap.add_argument("--steps", type=int, default=3, help="timed steps (one whole job each)")
    ap.add_argument("--warmup", type=int, default=1, help="untimed steps before the timed ones")
    ap.add_argument("--workload", default=WORKLOAD, help="plain workload a step runs (default: the benchmark job)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip timing the CPU oracle")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched, saturation, L=16 T=1, served and convergence legs")
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


def batched_leg():
    """Mixed (L, T) jobs (19 jobs, 4096 walkers, 10 iterations x 1000 sweeps):
    one persistent launch per iteration over every job (lock-step), in the
    default and in the autotuned batch shape; asynchronous lanes (jobs grouped
    by L, each group a batch on its own stream iterating on its own); and one
    plain launch per job.  The three batched modes run twice, in turn, and
    report the mean (one run varies by a few per cent)."""
    import torch

    from paper_1502_07214_amd import MucaBatch, MucaJob, autotune, workloads

    specs = workloads.batched_jobs()
    it, sw = workloads.BATCHED["iterations"], workloads.BATCHED["sweeps"]
    per_sweep = sum(n * L ** 3 for (L, T, n, s) in specs)
    tuned = autotune.tune_batch(specs, cache=autotune.CACHE, warm=autotune.BENCH_WARM_BATCH,
                                **autotune.BENCH_BATCH_PROBE)
    out = {"jobs": len(specs), "walkers": sum(n for (_, _, n, _) in specs), "iterations": it, "sweeps": sw,
           "attempts": per_sweep * it * sw, "tuned_shape": list(tuned), "lanes": list(workloads.BATCHED_LANES)}
    runs = {}
    for mode in ("batched", "batched_tuned", "async_lanes") * 2 + ("plain",):
        jobs = [MucaJob(L, T, n, seed=s, max_delta=1) for (L, T, n, s) in specs]
        batches = []
        if mode in ("batched", "batched_tuned"):
            batches = [MucaBatch(jobs)]
            if mode == "batched_tuned":
                batches[0].set_launch(*tuned)
        elif mode == "async_lanes":
            from paper_1502_07214_amd.serve import lane_of
            groups = {}
            for j in jobs:
                groups.setdefault(lane_of(j.L, workloads.BATCHED_LANES), []).append(j)
            for g in groups.values():
                st = torch.cuda.Stream()
                for j in g:
                    j.set_stream(st)
                batches.append(MucaBatch(g))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "async_lanes":
            left = {id(b): it for b in batches}
            for b in batches:
                b.submit(sw)
            while any(left.values()):
                moved = False
                for b in batches:
                    if left[id(b)] and b.poll():
                        for j in b.jobs:
                            j.update_weights(j.reduce_hist())
                        left[id(b)] -= 1
                        moved = True
                        if left[id(b)]:
                            b.submit(sw)
                if not moved:
                    time.sleep(2e-4)
        else:
            for k in range(it):
                if batches:
                    batches[0].sweep(sw)
                else:
                    for j in jobs:
                        j.sweep(sw)
                for j in jobs:
                    j.update_weights(j.reduce_hist())
        torch.cuda.synchronize()
        runs.setdefault(mode, []).append(time.perf_counter() - t0)
        dt = sum(runs[mode]) / len(runs[mode])
        out[mode + "_attempts_per_s"] = out["attempts"] / dt
        out[mode + "_s"] = dt
        out[mode + "_runs_s"] = list(runs[mode])
        for b in batches:
            b.free()
        for j in jobs:
            j.free()
    out["speedup"] = out["batched_attempts_per_s"] / out["plain_attempts_per_s"]
    out["async_vs_lockstep"] = out["async_lanes_attempts_per_s"] / out["batched_attempts_per_s"]
    return out


def served_leg():
    """The Poisson stream of MUCA jobs at its stated size (200 jobs, L 8..24,
    per-job Delta ranges): continuous batching in asynchronous lanes, the same
    in lock-step (one launch over every resident job per iteration), and one
    job at a time, each under the same wall budget (jobs unfinished by then
    are censored at it, so their latencies are lower bounds)."""
    from paper_1502_07214_amd import workloads
    from paper_1502_07214_amd.serve import ServeConfig, poisson_requests, serve, serve_plain

    sp = workloads.SERVED
    reqs = poisson_requests(sp["n_jobs"], sp["rate"], sp["seed"], sp["L_range"], sp["T_range"], sp["walker_choices"],
                            delta_halfwidth=sp["delta_halfwidth"])
    cfg = ServeConfig(sweeps=sp["sweeps"], threshold=sp["threshold"], max_iterations=sp["max_iterations"],
                      wall_budget=sp["wall_budget"], recursion=REC_ACC_EXT, lane_bounds=tuple(sp["lane_bounds"]),
                      entries_per_bin=sp["entries_per_bin"])
    out = {"spec": {k: v for k, v in sp.items()}, "recursion": "accumulated+extrapolate",
           "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))}
    modes = (("served_async", serve, cfg), ("served_lockstep", serve, dataclasses.replace(cfg, lane_bounds=())),
             ("one_at_a_time", serve_plain, cfg))
    for mode, fn, c in modes:
        print(f"[bench] served: {mode}", file=sys.stderr, flush=True)
        r = fn(reqs, c)
        out[mode] = {k: r[k] for k in ("jobs", "converged", "censored", "not_arrived", "makespan_s", "converged_per_s",
                                       "attempts_per_s", "latency_p50_s", "latency_p99_s",
                                       "latency_converged_p50_s", "latency_converged_p99_s", "iterations_p50",
                                       "long_iteration_jobs", "queue_depth_max")}
        if "host_s" in r:
            out[mode]["host_s"] = {k: round(v, 3) for k, v in r["host_s"].items()}
    return out


def c3_leg():
    """The L=16, T=1 (first-order regime), 1024-walker job in full (60
    iterations x 2*10^4 sweeps, 2*10^4 production sweeps, 200 Delta) in the
    autotuned launch shape, each iteration's sweep launch timed with HIP events
    on the job's stream; then the first iterations again in the library's
    default shape, for the same launches."""
    import numpy as np
    import torch

    from paper_1502_07214_amd import MucaJob, autotune, workloads

    w = workloads.workload("l16_t1_w1024")
    deltas = workloads.delta_grid(w["deltas"])
    shape = autotune.tune_job(w["L"], w["T"], w["n_walkers"], seed=w["seed"], probe_sweeps=1000,
                              cache=autotune.CACHE, warm=autotune.BENCH_WARM_PLAIN)
    per_launch = w["n_walkers"] * w["V"] * w["sweeps"]

    def run(launch, iterations, production):
        job = MucaJob(w["L"], w["T"], w["n_walkers"], seed=w["seed"], max_delta=len(deltas))
        if launch is not None:
            job.set_launch(*launch)
        used = job.get_launch()
        ms = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iterations):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(job.stream)
            job.sweep(w["sweeps"])
            e1.record(job.stream)
            job.update_weights(job.reduce_hist())
            ms.append(e0.elapsed_time(e1))
        if production:
            job.sweep(w["production"], record=True)
            job.reduce_hist()
            job.reweight(deltas)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        job.free()
        return used, ms, dt

    used, ms, dt = run(shape, w["iterations"], True)
    k = 6
    dused, dms, _ = run(None, k, False)
    launch_ms = float(np.mean(ms))
    rate = per_launch / (launch_ms * 1e-3)
    return {"workload": f"L={w['L']} T={w['T']} walkers={w['n_walkers']} {w['iterations']}x{w['sweeps']} + "
                        f"{w['production']} production, {len(deltas)} Delta",
            "tuned_shape": used, "attempts": w["attempts"], "seconds": dt, "attempts_per_s": w["attempts"] / dt,
            "sweep_launch_ms": launch_ms, "kernel_attempts_per_s": rate,
            "roofline_frac": rate * ALGO_SLOTS_PER_ATTEMPT / PEAK_SLOTS_PER_S,
            "roofline_frac_itemised": rate * ITEMISED_SLOTS_PER_ATTEMPT / PEAK_SLOTS_PER_S,
            "default_shape": dused, "first_launches": k,
            "default_first_ms": float(np.mean(dms)), "tuned_first_ms": float(np.mean(ms[:k])),
            "tuned_vs_default_first": float(np.mean(dms)) / float(np.mean(ms[:k]))}


def convergence_leg():
    """Iterations and seconds to a flat histogram (F > 0.5 over [0, V]) for
    single jobs: the plain recursion, edge extrapolation, and accumulated pair
    statistics with extrapolation, from a flat and from a tilted start."""
    import torch

    from paper_1502_07214_amd import MucaJob, workloads
    from paper_1502_07214_amd.serve import tilted_weights

    out = []
    for c in workloads.CONVERGENCE:
        for start in ("flat", "tilted"):
            for name, flags in (("plain", 0), ("extrapolate", REC_EXTRAPOLATE), ("accumulated+extrapolate", REC_ACC_EXT)):
                lnW = tilted_weights(c["L"], c["T"]) if start == "tilted" else None
                job = MucaJob(c["L"], c["T"], c["n_walkers"], seed=c["seed"], lnW=lnW, max_delta=1)
                job.set_recursion(flags)
                t0 = time.perf_counter()
                it, f = 0, 0.0
                while it < c["max_iterations"]:
                    job.sweep(c["sweeps"])
                    h = job.reduce_hist()
                    it += 1
                    f = job.update_weights(h)
                    if f > c["threshold"]:
                        break
                torch.cuda.synchronize()
                out.append({"L": c["L"], "T": c["T"], "walkers": c["n_walkers"], "sweeps": c["sweeps"],
                            "start": start, "recursion": name, "iterations": it, "flat": f > c["threshold"],
                            "seconds": time.perf_counter() - t0})
                job.free()
    return out


def saturation_run(L, T, n_walkers, seed, sweeps):
    """One saturation job: 10 untimed sweeps, then one launch of `sweeps`
    timed with HIP events on the job's stream, in the library's launch shape."""
    import torch

    from paper_1502_07214_amd import MucaJob

    job = MucaJob(L, T, n_walkers, seed=seed, max_delta=1)
    job.sweep(10)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    job.sweep(sweeps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    rate = n_walkers * L ** 3 * sweeps / (ms * 1e-3)
    shape = job.get_launch()
    job.free()
    return {"workload": f"L={L} T={T} walkers={n_walkers} sweeps={sweeps}", "launch": shape,
            "kernel_attempts_per_s": rate, "launch_ms": ms,
            "roofline_frac": rate * ALGO_SLOTS_PER_ATTEMPT / PEAK_SLOTS_PER_S,
            "roofline_frac_itemised": rate * ITEMISED_SLOTS_PER_ATTEMPT / PEAK_SLOTS_PER_S}


def saturation_leg():
    """The saturation job (L=8, 65 536 walkers), and the grid over L = 8, 12,
    16 and 1, 2, 4 waves of walkers per SIMD."""
    from paper_1502_07214_amd import workloads

    s = workloads.SATURATION
    out = saturation_run(s["L"], s["T"], s["n_walkers"], s["seed"], s["sweeps"])
    out["grid"] = [saturation_run(L, s["T"], n, s["seed"], s["sweeps"]) for (L, n) in workloads.SATURATION_GRID]
    return out


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
                      f"({t['attempts']:.3e} attempts, {dt:.1f} s)",
            "host": host_cpu()}


def host_cpu() -> str:
    """CPU model and logical CPU count of the host that timed the oracle."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical CPUs visible"



def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the walker-sharded multi-GPU path is a design, not code",
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
        "per_walker_attempts_per_s": kernel_rate / w["n_walkers"],
        "sweep_launch_ms": launch_ms,
        "final_flatness": flat,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS_PER_S / 1e12,
                     "unit": "Tslot/s", "frac": achieved / PEAK_SLOTS_PER_S,
                     "traffic": TRAFFIC_BYTES_PER_LAUNCH if shape == {"waves_per_walker": 4, "blocks_per_lane": 1,
                                                                      "lds_tables": 1, "packed": 0,
                                                                      "lds_bytes": 36960} else None,
                     "kernel": "muca_sweep_kernel", "slots_per_attempt": ALGO_SLOTS_PER_ATTEMPT,
                     "frac_itemised": kernel_rate * ITEMISED_SLOTS_PER_ATTEMPT / PEAK_SLOTS_PER_S,
                     "slots_per_attempt_itemised": ITEMISED_SLOTS_PER_ATTEMPT},
    }
    if not args.no_extra:
        print("[bench] batched leg", file=sys.stderr, flush=True)
        out["batched"] = batched_leg()
        print("[bench] saturation leg", file=sys.stderr, flush=True)
        out["saturation"] = saturation_leg()
        print("[bench] L=16 T=1 1024-walker leg", file=sys.stderr, flush=True)
        out["l16_t1_w1024"] = c3_leg()
        print("[bench] served leg", file=sys.stderr, flush=True)
        out["served"] = served_leg()
        print("[bench] convergence leg", file=sys.stderr, flush=True)
        out["convergence"] = convergence_leg()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, deltas)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
