"""Pins of the oracle's faster weight recursions (accumulated pair statistics,
edge extrapolation) against facts that do not come from the oracle itself:
special cases that reduce to the plain recursion, the harmonic weighting of
repeated identical statistics, exact linear continuations, and convergence to
the exactly known weights (L=2 enumeration, beta=0 closed form)."""
import math

import numpy as np
import pytest

import oracle
from tests import l2_exact

ACC, EXT = 1, 2


def fresh(L=2, T=1.0, flags=0, lnW=None):
    job = oracle.OracleJob(L, T, 1, seed=0, lnW=lnW)
    job.set_recursion(flags)
    return job


def rel(lnW):
    return np.asarray(lnW) - lnW[0]


def test_accumulated_first_iteration_is_the_plain_recursion():
    rng = np.random.default_rng(5)
    h = rng.integers(1, 10**6, size=28).astype(np.int64)
    lnW0 = rng.normal(size=28)
    a, p = fresh(3, flags=ACC, lnW=lnW0), fresh(3, flags=0, lnW=lnW0)
    fa, fp = a.update_weights(h), p.update_weights(h)
    assert fa == fp
    # same weights up to the constant the plain step removes from bin 0
    assert np.allclose(rel(a.lnW), rel(p.lnW), rtol=0, atol=1e-10)


def test_accumulated_repeats_average_harmonically():
    # the same histogram n times: the n-th step carries weight 1/n, so the
    # differences move by (1 + 1/2 + ... + 1/n) times the plain step
    h = np.array([5, 40, 7, 300, 2, 9, 11, 1000, 3], dtype=np.int64)
    job = fresh(2, flags=ACC)
    step = np.log(h[:-1].astype(float)) - np.log(h[1:].astype(float))
    for n in range(1, 6):
        job.update_weights(h)
        harmonic = sum(1.0 / m for m in range(1, n + 1))
        assert np.allclose(np.diff(job.lnW), harmonic * step, rtol=1e-12, atol=1e-12)


def test_accumulated_frontier_pairs_take_the_plain_step():
    h = np.array([0, 0, 50, 20, 0, 0, 0, 0, 0], dtype=np.int64)
    a, p = fresh(2, flags=ACC), fresh(2, flags=0)
    a.update_weights(h)
    p.update_weights(h)
    # visited bins and their empty neighbours move relative to each other as
    # in the plain recursion; pairs with no entries keep their difference
    assert np.allclose(np.diff(a.lnW)[1:4], np.diff(p.lnW)[1:4], rtol=0, atol=1e-12)
    assert np.diff(a.lnW)[0] == 0.0 and np.all(np.diff(a.lnW)[4:] == 0.0)


def test_flat_histogram_is_a_fixed_point():
    lnW = -l2_exact.ln_g_beta(0.5)
    for flags in (ACC, EXT, ACC | EXT):
        job = fresh(2, T=2.0, flags=flags, lnW=lnW)
        for _ in range(3):
            assert job.update_weights(np.full(9, 1234, dtype=np.int64)) == 1.0
        assert np.allclose(rel(job.lnW), rel(lnW), rtol=0, atol=1e-12)


def test_extrapolation_continues_linear_weights_exactly():
    V = 27
    s = 0.37
    lnW = 1.5 - s * np.arange(V + 1)
    h = np.zeros(V + 1, dtype=np.int64)
    h[9:17] = 1000  # flat inside [9, 16]: the recursion keeps the slope there
    for flags in (EXT, ACC | EXT):
        job = fresh(3, flags=flags, lnW=lnW)
        job.update_weights(h)
        # linear weights continue as the same line on both sides
        assert np.allclose(np.diff(job.lnW), -s, rtol=0, atol=1e-12)


def test_extrapolation_leaves_the_visited_range_alone():
    rng = np.random.default_rng(2)
    V = 27
    lnW = rng.normal(size=V + 1)
    h = np.zeros(V + 1, dtype=np.int64)
    h[5:20] = rng.integers(1, 100, size=15)
    p, e = fresh(3, flags=0, lnW=lnW), fresh(3, flags=EXT, lnW=lnW)
    p.update_weights(h)
    e.update_weights(h)
    assert np.array_equal(p.lnW[5:20], e.lnW[5:20])
    assert not np.allclose(p.lnW[20:], e.lnW[20:])


def test_visited_range_accumulates_over_iterations():
    V = 27
    h1 = np.zeros(V + 1, dtype=np.int64)
    h1[3:6] = 10
    h2 = np.zeros(V + 1, dtype=np.int64)
    h2[12:15] = 10
    job = fresh(3, flags=EXT)
    job.update_weights(h1)
    job.update_weights(h2)
    assert job.seen[3] == 1 and job.seen[14] == 1 and job.seen[8] == 0
    # bins inside [3, 14] that were never visited are not extrapolated
    before = job.lnW.copy()
    h3 = np.zeros(V + 1, dtype=np.int64)
    h3[4] = 1
    job.update_weights(h3)
    assert np.array_equal(job.lnW[5:15], before[5:15])


@pytest.mark.parametrize("flags", [ACC, ACC | EXT])
def test_variants_converge_to_exact_weights_l2(flags):
    beta = 0.5
    job = oracle.OracleJob(2, 1.0 / beta, 16, seed=4)
    job.set_recursion(flags)
    for it in range(25):
        job.sweep(4000)
        job.update_weights(job.take_hist())
    target = -l2_exact.ln_g_beta(beta)
    err = np.max(np.abs(np.diff(job.lnW) - np.diff(target)))
    assert err < 0.1, err


def test_variants_converge_to_beta0_density_of_states():
    # beta = 0: the flat-histogram weights are 1 / (C(V, E) 2^E) exactly
    L, V = 3, 27
    exact = np.array([-math.log(2.0 * (V - E + 1) / E) for E in range(1, V + 1)])
    for flags in (ACC, ACC | EXT):
        job = oracle.OracleJob(L, float("inf"), 16, seed=21)
        job.set_recursion(flags)
        for it in range(30):
            job.sweep(3000)
            flat = job.update_weights(job.take_hist())
        assert flat > 0.5
        diffs = np.diff(job.lnW)
        assert np.all(np.abs(diffs - exact) < 0.3), (flags, np.max(np.abs(diffs - exact)))


def iterations_to_flat(L, T, flags, sweeps, cap, seed=3, walkers=8, threshold=0.5):
    job = oracle.OracleJob(L, T, walkers, seed=seed)
    job.set_recursion(flags)
    for it in range(1, cap + 1):
        job.sweep(sweeps)
        if job.update_weights(job.take_hist()) > threshold:
            return it
    return cap + 1


def test_extrapolation_reaches_flatness_sooner():
    # L=4, T=2 from a flat start: the plain recursion must raise the far end
    # of the E_Delta range by ~3 beta V nats at <= ln(entries) per iteration
    plain = iterations_to_flat(4, 2.0, 0, 200, 60)
    fast = iterations_to_flat(4, 2.0, ACC | EXT, 200, 60)
    assert fast < plain, (fast, plain)


def test_accumulated_is_the_inverse_variance_mean_of_the_estimates():
    # each iteration estimates the flat-histogram difference as
    # d + log H(E) - log H(E+1); Poisson counts give that log-ratio the
    # variance 1/H(E) + 1/H(E+1), and the recursion keeps the mean of the
    # estimates weighted by the inverse variances
    rng = np.random.default_rng(9)
    lnW0 = rng.normal(size=9)
    hs = [rng.integers(1, 500, size=9).astype(np.int64) for _ in range(4)]
    job = fresh(2, flags=ACC, lnW=lnW0)
    num = np.zeros(8)
    den = np.zeros(8)
    for h in hs:
        d = np.diff(job.lnW)
        hf = h.astype(float)
        est = d + np.log(hf[:-1]) - np.log(hf[1:])
        w = 1.0 / (1.0 / hf[:-1] + 1.0 / hf[1:])
        num += w * est
        den += w
        job.update_weights(h)
        assert np.allclose(np.diff(job.lnW), num / den, rtol=0, atol=1e-10)


def test_accumulated_statistics_restart_when_a_visited_bin_is_missed():
    # after an iteration that leaves a bin unvisited between the lowest and
    # highest bins visited so far, the step is the plain one again: with K
    # restarted, each pair's weight k / K is 1 and the frontier pairs around
    # the missed bin take the plain step anyway
    h1 = np.array([0, 0, 30, 40, 50, 60, 0, 0, 0], dtype=np.int64)
    h2 = np.array([0, 0, 60, 10, 0, 20, 0, 0, 0], dtype=np.int64)
    a, p = fresh(2, flags=ACC), fresh(2, flags=0)
    for h in (h1, h2):
        a.update_weights(h)
        p.update_weights(h)
    assert np.allclose(np.diff(a.lnW)[1:7], np.diff(p.lnW)[1:7], rtol=0, atol=1e-12)
    # with the bin visited, the second histogram is averaged with the first
    h2c = np.array([0, 0, 60, 10, 5, 20, 0, 0, 0], dtype=np.int64)
    b, q = fresh(2, flags=ACC), fresh(2, flags=0)
    for h in (h1, h2c):
        b.update_weights(h)
        q.update_weights(h)
    assert not np.allclose(np.diff(b.lnW)[2:5], np.diff(q.lnW)[2:5])
    # a bin missed outside the visited range is no loss: 0 and 1 stay unseen
    h3 = np.array([0, 0, 60, 10, 5, 20, 0, 0, 0], dtype=np.int64)
    c = fresh(2, flags=ACC)
    for h in (h1, h3):
        c.update_weights(h)
    assert np.allclose(c.kacc[2:5], [h1[E] * h1[E + 1] / (h1[E] + h1[E + 1]) + h3[E] * h3[E + 1] / (h3[E] + h3[E + 1])
                                     for E in range(2, 5)], rtol=1e-15, atol=0)


def test_accumulated_statistics_restart_when_the_range_grows():
    # after an iteration that reaches a new bin, the next step is the plain
    # one again (the earlier estimates carry the bias of the missing range)
    h1 = np.array([0, 0, 30, 40, 50, 0, 0, 0, 0], dtype=np.int64)
    h2 = np.array([0, 0, 60, 10, 20, 5, 0, 0, 0], dtype=np.int64)
    a, p = fresh(2, flags=ACC), fresh(2, flags=0)
    for h in (h1, h2):
        a.update_weights(h)
        p.update_weights(h)
    assert np.allclose(np.diff(a.lnW)[1:6], np.diff(p.lnW)[1:6], rtol=0, atol=1e-12)
    # without growth the same second histogram is averaged with the first
    h2b = np.array([0, 0, 60, 10, 20, 0, 0, 0, 0], dtype=np.int64)
    b = fresh(2, flags=ACC)
    b.update_weights(h1)
    b.update_weights(h2b)
    assert not np.allclose(np.diff(b.lnW)[2:4], np.diff(p.lnW)[2:4])
