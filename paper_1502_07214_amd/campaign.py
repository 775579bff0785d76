"""Small-L campaign of the paper's observables (Sec. III at small sizes).

For each (L, T): weights converged to a flat E_Delta histogram (start tilted
towards the transition field, accumulated + extrapolating recursion unless the
point names another), a
production run recorded in time blocks, the peak of C(Delta) = d<E_J>/dDelta
with jackknife errors over the blocks, and at first-order temperatures the
equal-height field and barrier of the reweighted P(e_Delta).  Every step runs
through libmuca; this module sequences calls and picks brackets.

    python -m paper_1502_07214_amd.campaign            # the default points
    python -m paper_1502_07214_amd.campaign 8:1.0 12:2.0
    python -m paper_1502_07214_amd.campaign --walker-groups 8:1.0   # jackknife over walker groups
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

from . import analysis
from .muca import OBS_FIELDS, REC_ACCUMULATED, REC_EXTRAPOLATE, MucaJob, muca_flatness
from .serve import delta_mid, tilted_weights

_C = OBS_FIELDS.index("C_field")

# (L, T, walkers, sweeps per iteration, iteration cap, production blocks, sweeps per block
#  [, weight recursion flags; default accumulated + extrapolating])
# The default points are the small sizes at which the paper's fields are compared:
# the first-order fields at T = 1.0 and 0.9 (L = 8, 12) and the second-order shift
# at T = 2.0 (L = 8, 12, 16).  Command-line arguments pick among them.
POINTS = (
    (8, 1.0, 512, 1000, 1500, 8, 5000),
    (12, 1.0, 512, 2000, 1500, 8, 10000),
    (8, 0.9, 512, 1000, 1500, 8, 5000),
    (12, 0.9, 512, 2000, 1500, 8, 10000),
    (8, 2.0, 512, 1000, 600, 8, 5000),
    (12, 2.0, 512, 2000, 600, 8, 10000),
    (16, 2.0, 1024, 4000, 600, 8, 10000),
)
FIRST_ORDER_T = 1.4182  # below the tricritical temperature the transition is first order


def converge(job: MucaJob, sweeps: int, cap: int, threshold: float = 0.5, log=None) -> dict:
    """Iterate until the merged histogram is flat (min/mean > threshold on
    [0, V]) or the cap is reached; the weights are updated after every
    iteration that is not yet flat.  log(iteration, flatness) is called every
    50 iterations."""
    V = job.V
    f = 0.0
    it = 0
    while it < cap:
        job.sweep(sweeps)
        h = job.reduce_hist(reset=True)
        it += 1
        f = muca_flatness(h, 0, V)
        if log is not None and it % 50 == 0:
            log(it, f)
        if f > threshold:
            break
        job.update_weights(h)
    return {"iterations": it, "flatness": f, "flat": f > threshold}


def _bracket(grid: np.ndarray, values: np.ndarray):
    k = int(np.argmax(values))
    return float(grid[max(k - 1, 0)]), float(grid[min(k + 1, len(grid) - 1)]), k


def run_point(L: int, T: float, walkers: int, sweeps: int, cap: int, n_blocks: int, block_sweeps: int,
              recursion: int = REC_ACCUMULATED | REC_EXTRAPOLATE, seed: int = 0, grid=None, log=None,
              walker_groups: bool = False) -> dict:
    """One point: weights to a flat histogram, production, the peak of C(Delta)
    with jackknife errors and, below the tricritical temperature, the
    equal-height field and barrier.  The production is n_blocks x block_sweeps
    sweeps in consecutive time blocks, or (walker_groups) n_blocks x
    block_sweeps sweeps of every walker with the walkers split into n_blocks
    groups, the paper's independent runs."""
    t0 = time.perf_counter()
    dm = delta_mid(T)
    grid = np.linspace(dm - 1.0, dm + 0.5, 301) if grid is None else np.asarray(grid, dtype=np.float64)
    job = MucaJob(L, T, walkers, seed=seed, lnW=tilted_weights(L, T), max_delta=len(grid))
    job.set_recursion(recursion)
    out = {"L": L, "T": T, "walkers": walkers, "sweeps_per_iteration": sweeps, "recursion": recursion}
    out.update(converge(job, sweeps, cap, log=log))
    if walker_groups:
        blocks, total = analysis.walker_blocks(job, n_blocks, n_blocks * block_sweeps)
    else:
        blocks, total = analysis.production_blocks(job, n_blocks, block_sweeps)
    out["production_sweeps"] = n_blocks * block_sweeps
    out["blocks"] = "walker groups" if walker_groups else "time blocks"
    cs = job.reweight_sums(total, grid)[:, _C]
    lo, hi, k = _bracket(grid, cs)
    out["scan_peak_at_edge"] = k in (0, len(grid) - 1)
    if not out["scan_peak_at_edge"]:
        try:
            pk = analysis.jackknife_peak(job, blocks, total, lo, hi)
            out.update({"delta_star": pk["delta_star"], "delta_star_err": pk["delta_star_err"],
                        "C_star": pk["C_star"], "C_star_err": pk["C_star_err"]})
        except ValueError as e:  # a block subset without a maximum on the bracket
            out["peak_error"] = str(e)
    if T < FIRST_ORDER_T and "delta_star" in out:
        V = L ** 3
        lnP = job.reweight_hist(out["delta_star"])
        mid = lnP[int(0.2 * V):int(0.8 * V) + 1]
        split = int(0.2 * V) + int(np.argmin(np.where(np.isfinite(mid), mid, np.inf)))
        diffs = []
        for d in grid:
            p = job.reweight_hist(float(d))
            diffs.append(float(np.max(p[split:]) - np.max(p[:split])))
        diffs = np.array(diffs)
        cross = [i for i in range(len(grid) - 1) if diffs[i] > 0 and diffs[i + 1] < 0]
        if cross:
            i = cross[0]
            out["split_bin"] = split
            try:
                eq = analysis.jackknife_equal_height(job, blocks, total, float(grid[i]), float(grid[i + 1]), split)
                out.update({"delta_eqh": eq["delta_eqh"], "barrier": eq["barrier"],
                            "delta_eqh_err": eq["delta_eqh_err"], "barrier_err": eq["barrier_err"]})
            except ValueError as e:  # a block subset without a crossing on the bracket
                d_eqh, barrier = analysis.equal_height(job, float(grid[i]), float(grid[i + 1]), split)
                out.update({"delta_eqh": d_eqh, "barrier": barrier, "eqh_error": str(e)})
    out["seconds"] = time.perf_counter() - t0
    job.free()
    return out


def main(argv):
    pts = POINTS
    walker_groups = "--walker-groups" in argv
    argv = [a for a in argv if a != "--walker-groups"]
    if argv:
        want = [(int(a.split(":")[0]), float(a.split(":")[1])) for a in argv]
        pts = [p for p in POINTS if (p[0], p[1]) in want]
    for p in pts:
        print(f"[campaign] L={p[0]} T={p[1]}", file=sys.stderr, flush=True)
        log = lambda it, f: print(f"[campaign]   iteration {it}: flatness {f:.3f}", file=sys.stderr, flush=True)
        print(json.dumps(run_point(*p, log=log, walker_groups=walker_groups)), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
