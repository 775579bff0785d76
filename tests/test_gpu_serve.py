"""Serving loop: a job served in a Poisson mix (continuous batching) gives the
same iterations, flatness history, weights and final walker state as the same
job served alone, bit for bit."""
import dataclasses

import numpy as np
import pytest

from paper_1502_07214_amd.serve import Request, ServeConfig, serve, serve_plain, poisson_requests

pytestmark = pytest.mark.gpu


def test_served_equals_alone():
    reqs = poisson_requests(6, rate=200.0, seed=3, L_range=(4, 7), T_range=(0.9, 2.0),
                            walker_choices=(64, 128))
    print("[serve] requests", [(r.L, round(r.T, 3), r.n_walkers) for r in reqs], flush=True)
    cfg = ServeConfig(sweeps=40, threshold=0.5, max_iterations=30, max_walkers=256)
    mix = serve(reqs, cfg, keep_jobs=True)
    assert mix["jobs"] == 6
    for r in reqs[:3]:
        alone = serve_plain([dataclasses.replace(r, arrival=0.0)], cfg, keep_jobs=True)
        a, b = mix["records"][r.id], alone["records"][r.id]
        assert a.window == b.window
        assert a.iterations == b.iterations and a.flatness == b.flatness and a.converged == b.converged
        ja, jb = mix["jobs_kept"][r.id], alone["jobs_kept"][r.id]
        sa, sta = ja.read_state()
        sb, stb = jb.read_state()
        assert np.array_equal(sa, sb) and np.array_equal(sta, stb)
        assert ja.lnW.tobytes() == jb.lnW.tobytes()
        jb.free()
    for j in mix["jobs_kept"].values():
        j.free()


def test_admission_respects_capacity():
    reqs = poisson_requests(5, rate=1000.0, seed=4, L_range=(4, 5), walker_choices=(128,))
    cfg = ServeConfig(sweeps=20, threshold=0.5, max_iterations=5, max_walkers=256)
    out = serve(reqs, cfg)
    assert out["jobs"] == 5
    # at most two 128-walker jobs resident at once: the rest wait in the queue
    assert out["queue_depth_max"] >= 1
    recs = sorted(out["records"].values(), key=lambda r: r.admitted)
    for k in range(2, len(recs)):
        assert recs[k].admitted >= min(x.finished for x in recs[:k]) - 1e-9


def test_lone_and_batched_launches_alternate():
    """A slow stream: a job runs alone (its own launch) until the next one
    arrives, then in a batch, then alone again; its chain is the same as when
    it is served by itself."""
    reqs = [Request(0, 6, 1.0, 64, 11, 0.0), Request(1, 5, 2.0, 64, 12, 0.05), Request(2, 4, 1.4182, 64, 13, 0.1)]
    cfg = ServeConfig(sweeps=50, threshold=0.99, max_iterations=60, max_walkers=512)
    print("[serve] lone / batched alternation", flush=True)
    mix = serve(reqs, cfg, keep_jobs=True)
    assert mix["jobs"] == 3 and mix["censored"] == 3
    for r in reqs:
        alone = serve_plain([dataclasses.replace(r, arrival=0.0)], cfg, keep_jobs=True)
        a, b = mix["records"][r.id], alone["records"][r.id]
        assert a.iterations == b.iterations == 60 and a.flatness == b.flatness
        ja, jb = mix["jobs_kept"][r.id], alone["jobs_kept"][r.id]
        sa, sta = ja.read_state()
        sb, stb = jb.read_state()
        assert np.array_equal(sa, sb) and np.array_equal(sta, stb)
        assert ja.lnW.tobytes() == jb.lnW.tobytes()
        jb.free()
    for j in mix["jobs_kept"].values():
        j.free()


@pytest.mark.parametrize("lane_bounds", [(), (8, 17)])
def test_large_windowed_jobs_served_equal_alone(lane_bounds):
    """Jobs at L = 16..20 with Delta ranges Delta_mid(T) +- 0.1 (windows from
    the canonical probes), served in a mix of four, equal the same jobs served
    alone: window, flatness history, weights and walkers bit for bit; in
    lock-step and in asynchronous lanes (L <= 8, L <= 17, larger: three streams)."""
    reqs = [Request(0, 16, 0.95, 64, 101, 0.0, (2.85, 3.05)), Request(1, 20, 2.0, 64, 102, 0.0, (2.42, 2.62)),
            Request(2, 18, 1.4182, 128, 103, 0.01, (2.7446, 2.9446)), Request(3, 6, 1.2, 64, 104, 0.02, (2.8, 3.0)),
            Request(4, 12, 1.0, 64, 105, 0.0, (2.85, 3.05))]
    cfg = ServeConfig(sweeps=40, threshold=0.5, max_iterations=6, max_walkers=1024, lane_bounds=lane_bounds)
    print(f"[serve] windowed L=16..20 mix, lanes {lane_bounds}", flush=True)
    mix = serve(reqs, cfg, keep_jobs=True)
    assert mix["jobs"] == 5 and mix["lanes"] == len(lane_bounds) + 1
    for r in reqs[:3]:
        a = mix["records"][r.id]
        V = r.L ** 3
        assert 0 <= a.window[0] < a.window[1] <= V and a.window != (0, V)
        alone = serve_plain([dataclasses.replace(r, arrival=0.0)], cfg, keep_jobs=True)
        b = alone["records"][r.id]
        print(f"[serve] L={r.L} T={r.T} window {a.window} flatness {a.flatness[-1]:.3f}", flush=True)
        assert a.window == b.window and a.iterations == b.iterations and a.flatness == b.flatness
        ja, jb = mix["jobs_kept"][r.id], alone["jobs_kept"][r.id]
        assert ja.window == jb.window == a.window
        sa, sta = ja.read_state()
        sb, stb = jb.read_state()
        assert np.array_equal(sa, sb) and np.array_equal(sta, stb)
        assert ja.lnW.tobytes() == jb.lnW.tobytes()
        jb.free()
    for j in mix["jobs_kept"].values():
        j.free()


def test_long_iterations_served_equal_alone():
    """Iterations stretched once a job's histogram covers its window (here to
    about 120 entries per window bin: several launches of 40 sweeps per
    iteration) keep served == alone bit for bit, in asynchronous lanes, and
    a job that stretched its iterations merges only at their ends."""
    reqs = [Request(0, 6, 1.2, 64, 201, 0.0, (2.8, 3.0)), Request(1, 7, 2.0, 64, 202, 0.0, (2.42, 2.62)),
            Request(2, 8, 1.4182, 128, 203, 0.01, (2.7446, 2.9446)), Request(3, 10, 1.0, 64, 204, 0.02, (2.85, 3.05))]
    cfg = ServeConfig(sweeps=40, threshold=0.99, max_iterations=6, max_walkers=1024, lane_bounds=(7,),
                      entries_per_bin=120)
    print("[serve] stretched iterations, L=6..10 mix", flush=True)
    mix = serve(reqs, cfg, keep_jobs=True)
    assert any(a.span > 1 for a in mix["records"].values())
    assert mix["long_iteration_jobs"] == sum(1 for a in mix["records"].values() if a.span > 1)
    for r in reqs:
        a = mix["records"][r.id]
        alone = serve_plain([dataclasses.replace(r, arrival=0.0)], cfg, keep_jobs=True)
        b = alone["records"][r.id]
        print(f"[serve] L={r.L} window {a.window} span {a.span} iterations {a.iterations}", flush=True)
        assert (a.window, a.span, a.iterations, a.flatness) == (b.window, b.span, b.iterations, b.flatness)
        V = r.L ** 3
        assert a.attempts == b.attempts
        # attempts count every launch: (iterations before stretching) + span x (the rest)
        assert a.attempts % (r.n_walkers * V * cfg.sweeps) == 0
        ja, jb = mix["jobs_kept"][r.id], alone["jobs_kept"][r.id]
        sa, sta = ja.read_state()
        sb, stb = jb.read_state()
        assert np.array_equal(sa, sb) and np.array_equal(sta, stb)
        assert ja.lnW.tobytes() == jb.lnW.tobytes()
        jb.free()
    for j in mix["jobs_kept"].values():
        j.free()


def test_wall_budget_censors_unfinished_jobs():
    reqs = poisson_requests(4, rate=100.0, seed=5, L_range=(12, 12), walker_choices=(64,))
    cfg = ServeConfig(sweeps=200, threshold=0.99, max_iterations=10_000, wall_budget=1.5)
    out = serve(reqs, cfg)
    assert out["jobs"] == 4 and out["converged"] == 0 and out["censored"] == 4
    assert all(abs(r.finished - 1.5) < 1e-9 for r in out["records"].values())
    plain = serve_plain(reqs, cfg)
    assert plain["censored"] == 4 and plain["jobs"] == 4


def test_batch_submit_poll_finish():
    """muca_batch_submit returns at once; poll turns true when the launch has
    finished; the results equal a synchronous batched sweep."""
    from paper_1502_07214_amd import MucaBatch, MucaJob

    specs = [(8, 1.0, 64, 7), (12, 2.0, 32, 8)]
    a = [MucaJob(L, T, n, seed=s, max_delta=1) for (L, T, n, s) in specs]
    b = [MucaJob(L, T, n, seed=s, max_delta=1) for (L, T, n, s) in specs]
    ba, bb = MucaBatch(a), MucaBatch(b)
    ba.submit(400)
    polls = 0
    while not ba.poll():
        polls += 1
    ba.finish()
    bb.sweep(400)
    for x, y in zip(a, b):
        assert np.array_equal(x.reduce_hist(), y.reduce_hist())
        assert np.array_equal(x.read_state()[1], y.read_state()[1])
    print(f"[serve] submit/poll: {polls} polls before done", flush=True)
    ba.free()
    bb.free()
    for j in a + b:
        j.free()
