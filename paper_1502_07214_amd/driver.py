"""Plain parallel-MUCA job driver over the libmuca ABI (Sec. II of the paper).

One iteration = every walker sweeps `sweeps` times under the current weights
(muca_sweep), the walkers' E_Delta histograms are merged (muca_reduce_hist) and
the weights are updated by the recursion (muca_update_weights).  After the
iterations a production run records the per-bin sums and the job is reweighted
to a Delta grid (muca_reweight).  This module only sequences ABI calls.
"""
from __future__ import annotations

import numpy as np

from .muca import MucaJob


def run_iterations(job: MucaJob, iterations: int, sweeps: int, trace: bool = False,
                   stop_flatness: float = None) -> dict:
    hists, flats, lnws = [], [], []
    for it in range(iterations):
        job.sweep(sweeps)
        h = job.reduce_hist(reset=True)
        f = job.update_weights(h)
        flats.append(f)
        if trace:
            hists.append(h)
            lnws.append(job.lnW)
        if stop_flatness is not None and f > stop_flatness:
            break
    return {"hists": hists, "flatness": flats, "lnW": lnws}


def run_plain(job: MucaJob, iterations: int, sweeps: int, production: int, deltas, trace: bool = False) -> dict:
    out = run_iterations(job, iterations, sweeps, trace=trace)
    job.sweep(production, record=True)
    out["production_hist"] = job.reduce_hist(reset=True)
    out["obs"] = job.reweight(np.asarray(deltas, dtype=np.float64))
    return out
