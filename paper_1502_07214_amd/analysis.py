"""Analysis of a multicanonical production run (Sec. II-III of the paper).

* Pseudo-critical point: Delta*_L maximises C(Delta) = d<E_J>/dDelta; it is
  located by bisection on the zero of dC/dDelta (the second field derivative of
  <E_J>), each evaluation a reweighting on the device.  C*_L = C(Delta*_L).
* Jackknife: the production run is recorded in w blocks, either consecutive
  time blocks or groups of walkers (the paper's independent production runs:
  each group's chains are independent of the others'); the estimate is
  repeated on the w subsets that each leave one block out, and the error is
  sqrt((w-1)/w sum (x_j - mean)^2).
* Equal-height field: the Delta where the two peaks of the reweighted P(e_Delta)
  (maxima below and above a split bin) have equal height; the barrier
  ln(P_max / P_min) / (2 beta Delta_eqh) uses the minimum of P between them.

Every reweighting runs in libmuca (muca_reweight, muca_reweight_sums,
muca_reweight_hist); this module only drives the searches.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from .muca import OBS_FIELDS, MucaBatch, MucaJob

_DC = OBS_FIELDS.index("dC_dDelta")
_C = OBS_FIELDS.index("C_field")


def _reweight(job: MucaJob, sums, d: float) -> np.ndarray:
    return (job.reweight([d]) if sums is None else job.reweight_sums(sums, [d]))[0]


def peak(job: MucaJob, lo: float, hi: float, tol: float = 1e-11, sums=None) -> Tuple[float, float]:
    """(Delta*, C*) in [lo, hi]; dC/dDelta must go from + at lo to - at hi."""
    f_lo, f_hi = _reweight(job, sums, lo)[_DC], _reweight(job, sums, hi)[_DC]
    if not (f_lo > 0 and f_hi < 0):
        raise ValueError("dC/dDelta does not change sign from + to - on the bracket")
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if _reweight(job, sums, mid)[_DC] > 0:
            lo = mid
        else:
            hi = mid
    d = 0.5 * (lo + hi)
    return d, float(_reweight(job, sums, d)[_C])


def _zero_sums(V: int) -> dict:
    return {k: [0] * (V + 1) for k in ("H", "SJ", "SJJ", "SA", "SM2", "SM4")} | {"V": V}


def _minus(a: dict, b: dict) -> dict:
    return {k: ([x - y for x, y in zip(a[k], b[k])] if k != "V" else a[k]) for k in a}


def production_blocks(job: MucaJob, n_blocks: int, sweeps: int) -> Tuple[List[dict], dict]:
    """Record n_blocks consecutive production segments of `sweeps` sweeps;
    return the per-block per-bin sums and their total (exact integers)."""
    job.reset_accum()
    prev = _zero_sums(job.V)
    blocks = []
    for _ in range(n_blocks):
        job.sweep(sweeps, record=True)
        cur = job.read_accum()
        blocks.append(_minus(cur, prev))
        prev = cur
    return blocks, prev


def walker_blocks(job: MucaJob, n_groups: int, sweeps: int) -> Tuple[List[dict], dict]:
    """Record a production run of `sweeps` sweeps per group of walkers: the
    job's walkers are split into n_groups contiguous ranges, each swept (in
    one batched launch) as a sub-job holding that range (the same seed,
    weights and window, so every walker runs its own chain of the job).
    Afterwards the job holds the walkers' final states and the total sums,
    as after reset_accum() and sweep(sweeps, record=True); its iteration
    histogram is left as it was.  Returns the per-group sums and their total."""
    if not 1 <= n_groups <= job.n_walkers:
        raise ValueError("n_groups must lie in 1..n_walkers")
    spins, state = job.read_state()
    lo, hi = job.window
    edges = [job.n_walkers * g // n_groups for g in range(n_groups + 1)]
    weights = job.lnW
    subs, batch = [], None
    try:
        for g in range(n_groups):
            a, b = edges[g], edges[g + 1]
            sub = MucaJob(job.L, job.T, b - a, seed=job.seed, lnW=weights, max_delta=1, device=job.device,
                          first_walker=job.first_walker + a)
            subs.append(sub)
            if (lo, hi) != (0, job.V):
                sub.set_window(lo, hi)
            sub.write_state(spins[a:b], state[a:b])
        batch = MucaBatch(subs)
        batch.sweep(sweeps, record=True)
        blocks = [sub.read_accum() for sub in subs]
        finals = [sub.read_state() for sub in subs]
    finally:
        if batch is not None:
            batch.free()
        for sub in subs:
            sub.free()
    total = _zero_sums(job.V)
    for blk in blocks:
        total = {k: ([x + y for x, y in zip(total[k], blk[k])] if k != "V" else total[k]) for k in total}
    job.write_state(np.concatenate([f[0] for f in finals]), np.concatenate([f[1] for f in finals]))
    job.write_accum(total)
    return blocks, total


def jackknife(values) -> Tuple[float, float]:
    v = np.asarray(values, dtype=np.float64)
    w = len(v)
    m = float(v.mean())
    return m, float(math.sqrt((w - 1) / w * np.sum((v - m) ** 2)))


def jackknife_peak(job: MucaJob, blocks: List[dict], total: dict, lo: float, hi: float, tol: float = 1e-11):
    """Delta*, C* on all measurements, with jackknife errors over the blocks."""
    d, c = peak(job, lo, hi, tol, sums=total)
    loo = [peak(job, lo, hi, tol, sums=_minus(total, b)) for b in blocks]
    dj, de = jackknife([x[0] for x in loo])
    cj, ce = jackknife([x[1] for x in loo])
    return {"delta_star": d, "C_star": c, "delta_star_err": de, "C_star_err": ce,
            "delta_star_jk_mean": dj, "C_star_jk_mean": cj, "blocks": len(blocks)}


def _peaks(lnP: np.ndarray, split: int):
    a = int(np.argmax(lnP[:split]))
    b = split + int(np.argmax(lnP[split:]))
    return a, float(lnP[a]), b, float(lnP[b])


def _log_hist(job: MucaJob, hist, d: float) -> np.ndarray:
    return job.reweight_hist(d) if hist is None else job.reweight_hist_sums(hist, d)


def equal_height(job: MucaJob, lo: float, hi: float, split: int, tol: float = 1e-11,
                 hist=None) -> Tuple[float, float]:
    """(Delta_eqh, barrier) with Delta_eqh in [lo, hi], from the production
    histogram or, when given, from hist (V+1 counts under the job's weights)."""
    def diff(d):
        _, a, _, b = _peaks(_log_hist(job, hist, d), split)
        return b - a
    if not (diff(lo) > 0 and diff(hi) < 0):
        raise ValueError("peak heights do not cross on the bracket")
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if diff(mid) > 0:
            lo = mid
        else:
            hi = mid
    d = 0.5 * (lo + hi)
    lnP = _log_hist(job, hist, d)
    e1, p1, e2, p2 = _peaks(lnP, split)
    pmin = float(np.min(lnP[e1:e2 + 1]))
    barrier = (max(p1, p2) - pmin) / (2.0 * job.beta * d) if job.beta > 0 and d != 0 else float("nan")
    return d, barrier


def jackknife_equal_height(job: MucaJob, blocks: List[dict], total: dict, lo: float, hi: float, split: int,
                           tol: float = 1e-11):
    """Delta_eqh and the barrier on all measurements, with jackknife errors
    over the production blocks (each leave-one-out histogram reweighted on
    the device)."""
    d, b = equal_height(job, lo, hi, split, tol, hist=total["H"])
    loo = [equal_height(job, lo, hi, split, tol, hist=[x - y for x, y in zip(total["H"], blk["H"])])
           for blk in blocks]
    dj, de = jackknife([x[0] for x in loo])
    bj, be = jackknife([x[1] for x in loo])
    return {"delta_eqh": d, "barrier": b, "delta_eqh_err": de, "barrier_err": be,
            "delta_eqh_jk_mean": dj, "barrier_jk_mean": bj, "blocks": len(blocks)}
