"""Host-side sequencing that needs no GPU: request streams, transition fields,
tilted starts, the jackknife, the campaign's convergence loop and brackets, the
batched job table, the serving summary, and the library's host-only flatness
measure."""
import math
import os

import numpy as np
import pytest

from paper_1502_07214_amd import analysis, campaign, serve, workloads
from paper_1502_07214_amd.muca import muca_flatness
from paper_1502_07214_amd.serve import TRANSITION, delta_mid, poisson_requests, tilted_weights


def test_delta_mid_hits_the_paper_fields_and_interpolates():
    for T, d in TRANSITION:
        assert delta_mid(T) == d
    (t0, d0), (t1, d1) = TRANSITION[1], TRANSITION[2]
    assert delta_mid(0.5 * (t0 + t1)) == pytest.approx(0.5 * (d0 + d1), rel=1e-15)
    # outside the tabulated range the end values hold
    assert delta_mid(0.5) == TRANSITION[0][1] and delta_mid(3.0) == TRANSITION[-1][1]


def test_tilted_weights_are_the_canonical_ensemble_at_delta_mid():
    L, T = 5, 1.2
    w = tilted_weights(L, T)
    assert w.shape == (L ** 3 + 1,) and w[0] == 0.0
    # exp(lnW(E+1) - lnW(E)) = exp(-beta Delta_mid): the Boltzmann factor of one more occupied site
    assert np.allclose(np.diff(w), -delta_mid(T) / T, rtol=1e-13, atol=0)


def test_poisson_requests_are_seeded_and_well_formed():
    a = poisson_requests(500, 20.0, seed=3, L_range=(8, 24), walker_choices=(64, 128))
    b = poisson_requests(500, 20.0, seed=3, L_range=(8, 24), walker_choices=(64, 128))
    assert [(r.L, r.T, r.n_walkers, r.seed, r.arrival) for r in a] == [(r.L, r.T, r.n_walkers, r.seed, r.arrival) for r in b]
    arr = np.array([r.arrival for r in a])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    assert {r.L for r in a} <= set(range(8, 25)) and {r.n_walkers for r in a} <= {64, 128}
    assert all(0.9 <= r.T <= 2.0 for r in a)
    assert len({r.seed for r in a}) == len(a)
    # exponential gaps: the mean gap of 20000 arrivals is within 3 % of 1/rate
    many = poisson_requests(20000, 20.0, seed=1)
    gaps = np.diff([r.arrival for r in many])
    assert abs(gaps.mean() * 20.0 - 1.0) < 0.03


def test_jackknife_of_leave_one_out_means_is_the_standard_error():
    rng = np.random.default_rng(7)
    x = rng.normal(size=12)
    loo = [(x.sum() - xi) / (len(x) - 1) for xi in x]
    m, e = analysis.jackknife(loo)
    assert m == pytest.approx(x.mean(), rel=1e-12)
    assert e == pytest.approx(x.std(ddof=1) / math.sqrt(len(x)), rel=1e-12)


def test_block_sums_subtract_exactly():
    a = {"H": [5, 7], "SJ": [2 ** 62, -3], "V": 1}
    b = {"H": [1, 7], "SJ": [2 ** 62 - 1, -4], "V": 1}
    assert analysis._minus(a, b) == {"H": [4, 0], "SJ": [1, 1], "V": 1}


def test_bracket_around_the_scan_maximum():
    g = np.linspace(0.0, 1.0, 11)
    assert campaign._bracket(g, -(g - 0.3) ** 2) == (0.2, 0.4, 3)
    assert campaign._bracket(g, g) == (0.9, 1.0, 10)  # maximum at the edge: bracket clipped
    assert campaign._bracket(g, -g) == (0.0, 0.1, 0)


class _FakeJob:
    """Stands in for MucaJob in the convergence loop: hands out a fixed
    sequence of histograms and records the updates it is asked for."""

    def __init__(self, V, hists):
        self.V, self.hists, self.updates, self.sweeps = V, list(hists), [], 0

    def sweep(self, n):
        self.sweeps += n

    def reduce_hist(self, reset=True):
        return np.asarray(self.hists.pop(0), dtype=np.int64)

    def update_weights(self, h):
        self.updates.append(h.copy())


def test_converge_stops_at_the_first_flat_iteration():
    V = 3
    rough, flat = [1, 9, 9, 9], [6, 5, 7, 6]
    job = _FakeJob(V, [rough, rough, flat, rough])
    out = campaign.converge(job, sweeps=10, cap=10)
    assert out == {"iterations": 3, "flatness": muca_flatness(np.array(flat), 0, V), "flat": True}
    assert len(job.updates) == 2 and job.sweeps == 30  # no update after the flat one


def test_converge_respects_the_cap():
    job = _FakeJob(2, [[0, 4, 4]] * 5)
    out = campaign.converge(job, sweeps=1, cap=5)
    assert out["iterations"] == 5 and not out["flat"] and len(job.updates) == 5


def test_batched_workload_table():
    jobs = workloads.batched_jobs()
    spec = workloads.BATCHED
    assert sum(n for (_, _, n, _) in jobs) == spec["groups"] * spec["group_walkers"]
    assert all(n % spec["group_walkers"] == 0 for (_, _, n, _) in jobs)
    assert len({(L, T) for (L, T, _, _) in jobs}) == len(jobs)  # one job per (L, T)
    assert all(L in spec["Ls"] and T in spec["Ts"] for (L, T, _, _) in jobs)
    assert len({s for (_, _, _, s) in jobs}) == len(jobs)
    assert jobs == workloads.batched_jobs()


@pytest.mark.parametrize("lo,hi", [(0, 9), (2, 5), (4, 4)])
def test_host_flatness_is_min_over_mean(lo, hi):
    h = np.array([3, 8, 5, 9, 4, 7, 6, 2, 10, 1], dtype=np.int64)
    w = h[lo:hi + 1]
    assert muca_flatness(h, lo, hi) == pytest.approx(w.min() / w.mean(), rel=1e-15)
    assert muca_flatness(np.zeros(10, dtype=np.int64), lo, hi) == 0.0


def test_lanes_split_jobs_by_lattice_size():
    """Lane k holds L <= bounds[k] (and above the previous bound); the last
    lane everything larger; no bounds: one lane."""
    b = (12, 16, 20)
    assert [serve.lane_of(L, b) for L in (8, 12, 13, 16, 17, 20, 21, 24)] == [0, 0, 1, 1, 2, 2, 3, 3]
    assert serve.lane_of(24, ()) == 0


def test_iteration_span_waits_for_coverage_then_counts_entries():
    """One launch per iteration until every bin of the window was visited;
    then enough launches for entries_per_bin entries per window bin (rounded
    up); entries_per_bin 0 keeps one launch."""
    h = np.zeros(101, dtype=np.int64)
    h[10:61] = 5
    h[30] = 0
    assert serve.iteration_span(h, 10, 60, 64, 500, 200) == 1      # a bin of the window unvisited
    h[30] = 1
    assert serve.iteration_span(h, 10, 60, 64, 500, 200) == 1      # 51 bins x 200 < 64 x 500
    assert serve.iteration_span(h, 10, 60, 8, 100, 200) == 13      # ceil(51 x 200 / 800)
    assert serve.iteration_span(h, 10, 60, 8, 100, 0) == 1
    assert serve.iteration_span(h, 0, 100, 8, 100, 200) == 1       # bins outside the visited range
    h[:] = 1
    assert serve.iteration_span(h, 0, 100, 1, 1, 3) == 303


def test_iteration_span_counts_earlier_coverage_for_short_launches():
    """A launch with fewer than ln B + 3 entries per window bin (B bins) often
    leaves bins empty even under flat weights; there the bins that earlier
    iterations visited count towards coverage.  Longer launches still need
    one iteration that covers the window."""
    B = 5000
    h = np.ones(B + 1, dtype=np.int64)
    h[100] = 0                                   # this iteration missed a bin
    seen = np.ones(B + 1, dtype=bool)            # an earlier one visited it
    # 64 x 500 = 32 000 entries < 5001 x (ln 5001 + 3) = 57 600: counts seen
    assert serve.iteration_span(h, 0, B, 64, 500, 200) == 1
    assert serve.iteration_span(h, 0, B, 64, 500, 200, seen=seen) == 32   # ceil(5001 x 200 / 32 000)
    seen[200] = False
    assert serve.iteration_span(h, 0, B, 64, 500, 200, seen=seen) == 1
    seen[200] = True
    # 128 x 500 = 64 000 entries > 57 600: one iteration must cover the window
    assert serve.iteration_span(h, 0, B, 128, 500, 200, seen=seen) == 1
    h[100] = 1
    assert serve.iteration_span(h, 0, B, 128, 500, 200, seen=seen) == 16  # ceil(5001 x 200 / 64 000)


def test_serve_summary_separates_censored_jobs():
    from paper_1502_07214_amd.serve import JobRecord, Request, _summary
    recs = {}
    for i, (lat, conv) in enumerate([(1.0, True), (2.0, True), (3.0, True), (50.0, False)]):
        r = JobRecord(Request(i, 8, 1.0, 64, i, 0.0), admitted=0.0, finished=lat, iterations=10, converged=conv)
        recs[i] = r
    out = _summary(recs, makespan=50.0, attempts=100, launches=4, depth=[0, 2, 1], kept={})
    assert out["converged"] == 3 and out["censored"] == 1
    assert out["latency_p99_s"] == pytest.approx(np.percentile([1, 2, 3, 50], 99))
    assert out["latency_converged_p99_s"] == pytest.approx(np.percentile([1, 2, 3], 99))
    assert out["latency_converged_p50_s"] == 2.0 and out["queue_depth_max"] == 2


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: asked for more it prints one JSON line
    saying so and exits with status 2, before touching the device."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
