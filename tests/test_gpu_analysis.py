"""Analysis on the GPU path vs the oracle on the same (bit-identical) chains:
reweighted ln P(E_Delta), the peak of C(Delta) with jackknife errors over time
blocks, and the equal-height field with its barrier."""
import numpy as np
import pytest

import oracle
from paper_1502_07214_amd import MucaJob, analysis

pytestmark = pytest.mark.gpu


def make_pair(L, T, nw, seed, iterations, sweeps, lnW=None):
    job = MucaJob(L, T, nw, seed=seed, lnW=lnW, max_delta=4)
    o = oracle.OracleJob(L, T, nw, seed, lnW=lnW)
    for _ in range(iterations):
        job.sweep(sweeps)
        job.update_weights(job.reduce_hist())
        o.sweep(sweeps)
        o.update_weights(o.take_hist())
    assert job.lnW.tobytes() == o.lnW.tobytes()
    return job, o


def oracle_blocks(o, n_blocks, sweeps):
    o.reset_accum()
    prev = {k: [0] * (o.V + 1) for k in ("H", "SJ", "SJJ", "SA", "SM2", "SM4")} | {"V": o.V}
    blocks = []
    for _ in range(n_blocks):
        o.sweep(sweeps, record=True)
        cur = o.bin_sums()
        blocks.append(oracle.block_sums_difference(cur, prev))
        prev = cur
    return blocks, prev


def test_peak_and_jackknife_match_oracle():
    L, T = 4, 1.4182
    print(f"[analysis] peak L={L} T={T}", flush=True)
    job, o = make_pair(L, T, 16, 21, 8, 1000)
    blocks, total = analysis.production_blocks(job, 4, 1000)
    oblocks, ototal = oracle_blocks(o, 4, 1000)
    assert total == ototal and blocks == oblocks
    # bracket the maximum of C from a scan of the oracle
    grid = np.linspace(1.5, 4.0, 126)
    cs = oracle.reweight(o.V, o.beta, o.lnW, ototal, grid)[:, oracle.OBS_FIELDS.index("C_field")]
    k = int(np.argmax(cs))
    lo, hi = grid[max(k - 2, 0)], grid[min(k + 2, len(grid) - 1)]
    d_o, c_o = oracle.peak(o.V, o.beta, o.lnW, ototal, lo, hi)
    d_g, c_g = analysis.peak(job, lo, hi, sums=total)
    assert abs(d_g - d_o) < 1e-9 and abs(c_g - c_o) < 1e-10 * abs(c_o)
    jk = analysis.jackknife_peak(job, blocks, total, lo, hi)
    loo = [oracle.peak(o.V, o.beta, o.lnW, oracle.block_sums_difference(ototal, b), lo, hi) for b in oblocks]
    dm, de = oracle.jackknife([x[0] for x in loo])
    cm, ce = oracle.jackknife([x[1] for x in loo])
    assert abs(jk["delta_star"] - d_o) < 1e-9
    assert abs(jk["delta_star_err"] - de) < 1e-8 * max(de, 1e-3)
    assert abs(jk["C_star_err"] - ce) < 1e-8 * max(ce, 1e-3)
    # the device reweighting of the job's own sums agrees with the sums path
    assert np.array_equal(job.reweight([d_g]), job.reweight_sums(total, [d_g]))
    job.free()


def test_log_hist_and_equal_height_match_oracle():
    L, T = 4, 1.0
    print(f"[analysis] equal height L={L} T={T}", flush=True)
    # start tilted towards the transition field Delta* = 2.944 the paper gives at T = 1
    job, o = make_pair(L, T, 16, 22, 10, 1000, lnW=-(1.0 / T) * 2.944 * np.arange(L ** 3 + 1))
    job.reset_accum()
    job.sweep(3000, record=True)
    o.reset_accum()
    o.sweep(3000, record=True)
    H = o.bin_sums()["H"]
    for d in (2.5, 2.9, 3.1):
        g = job.reweight_hist(d)
        r = oracle.reweighted_log_hist(o.V, o.beta, o.lnW, H, d)
        fin = np.isfinite(r)
        assert np.array_equal(fin, np.isfinite(g))
        assert np.all(np.abs(g[fin] - r[fin]) <= 1e-12 * np.maximum(1.0, np.abs(r[fin])))
    split = o.V // 2
    grid = np.linspace(2.0, 4.0, 81)
    diffs = []
    for d in grid:
        _, a, _, b = oracle.two_peaks(oracle.reweighted_log_hist(o.V, o.beta, o.lnW, H, d), split)
        diffs.append(b - a)
    k = next(i for i in range(len(grid) - 1) if diffs[i] > 0 and diffs[i + 1] < 0)
    d_o, b_o = oracle.equal_height(o.V, o.beta, o.lnW, H, grid[k], grid[k + 1], split)
    d_g, b_g = analysis.equal_height(job, grid[k], grid[k + 1], split)
    assert abs(d_g - d_o) < 1e-9
    assert abs(b_g - b_o) < 1e-9 * max(1.0, abs(b_o))
    job.free()


def test_equal_height_closed_form_on_device():
    """The device reweighting of a histogram whose reweighted distribution is
    known in closed form (Sec. II): H(E) integer counts recorded under weights
    lnW(E) = ln H(E) - g(E) - beta D0 E, g the symmetric quartic double well
    -a((E - c)^2 - s^2)^2 / s^4 about c = V/2 with peaks at c +- s.  Then
    ln P(E; Delta) = g(E) - beta (Delta - D0) E + const, so the two peaks are
    equal at D0 and the barrier of Sec. III is a / (2 beta D0), independently of
    the oracle's code."""
    L, T, D0, a, s = 4, 0.9, 2.964, 7.5, 12
    V, beta = L ** 3, 1.0 / 0.9
    print(f"[analysis] closed-form equal height L={L} T={T}", flush=True)
    E = np.arange(V + 1, dtype=np.float64)
    g = -a * ((E - V / 2) ** 2 - s * s) ** 2 / s ** 4
    rng = np.random.default_rng(11)
    H = rng.integers(10 ** 9, 10 ** 12, size=V + 1).astype(np.int64)
    lnW = np.log(H.astype(np.float64)) - g - beta * D0 * E
    job = MucaJob(L, T, 1, seed=0, lnW=lnW, max_delta=1)
    d, b = analysis.equal_height(job, D0 - 0.05, D0 + 0.05, V // 2, hist=H)
    assert abs(d - D0) < 1e-9
    assert abs(b - a / (2.0 * beta * D0)) < 1e-9 * a / (2.0 * beta * D0)
    lnP = job.reweight_hist_sums(H, D0)
    assert np.all(np.abs((lnP - lnP.max()) - g) < 1e-9 * np.maximum(1.0, np.abs(g)))
    job.free()


@pytest.mark.parametrize("T", [1.0, 1.6])
def test_peak_on_device_matches_exact_l2(T):
    """Delta* (the maximum of C(Delta), Sec. III) from the device reweighting of
    the exact L = 2 expected per-bin sums (scaled to 10^12 measurements and
    rounded to integers) against the enumeration: at Delta* the exact
    dC/dDelta vanishes and C* equals the exact C there."""
    from tests import l2_exact

    beta = 1.0 / T
    lnW = -l2_exact.ln_g_beta(beta)
    ex = l2_exact.muca_bin_sums(beta, lnW, n=1e12)
    sums = {k: [int(round(v)) for v in ex[k]] for k in ("H", "SJ", "SJJ", "SA", "SM2", "SM4")} | {"V": 8}
    job = MucaJob(2, T, 1, seed=0, lnW=lnW, max_delta=1)
    d, c = analysis.peak(job, 2.0, 4.0, sums=sums)
    exact = l2_exact.canonical(beta, d)
    assert abs(exact["dC_dDelta"]) < 1e-8 * max(1.0, abs(exact["C_field"]))
    assert abs(c - exact["C_field"]) < 1e-9 * abs(exact["C_field"])
    job.free()


def test_jackknife_equal_height_matches_oracle():
    """Jackknife of the equal-height field and barrier over production blocks:
    every leave-one-out histogram reweighted on the device, against the
    oracle's reweighting of the same (bit-identical) blocks."""
    L, T = 4, 1.0
    print(f"[analysis] jackknife equal height L={L} T={T}", flush=True)
    job, o = make_pair(L, T, 16, 23, 10, 1000, lnW=-(1.0 / T) * 2.944 * np.arange(L ** 3 + 1))
    blocks, total = analysis.production_blocks(job, 4, 1500)
    oblocks, ototal = oracle_blocks(o, 4, 1500)
    assert total == ototal and blocks == oblocks
    split = o.V // 2
    grid = np.linspace(2.0, 4.0, 81)
    diffs = []
    for d in grid:
        _, a, _, b = oracle.two_peaks(oracle.reweighted_log_hist(o.V, o.beta, o.lnW, ototal["H"], d), split)
        diffs.append(b - a)
    k = next(i for i in range(len(grid) - 1) if diffs[i] > 0 and diffs[i + 1] < 0)
    lo, hi = grid[max(k - 1, 0)], grid[min(k + 2, len(grid) - 1)]
    jk = analysis.jackknife_equal_height(job, blocks, total, lo, hi, split)
    loo = [oracle.equal_height(o.V, o.beta, o.lnW, [x - y for x, y in zip(ototal["H"], b["H"])], lo, hi, split)
           for b in oblocks]
    d_o, b_o = oracle.equal_height(o.V, o.beta, o.lnW, ototal["H"], lo, hi, split)
    assert abs(jk["delta_eqh"] - d_o) < 1e-9 and abs(jk["barrier"] - b_o) < 1e-9 * max(1.0, b_o)
    de = oracle.jackknife([x[0] for x in loo])[1]
    be = oracle.jackknife([x[1] for x in loo])[1]
    assert abs(jk["delta_eqh_err"] - de) < 1e-6 * max(de, 1e-6)
    assert abs(jk["barrier_err"] - be) < 1e-6 * max(be, 1e-6)
    job.free()


@pytest.mark.parametrize("window", [None, (20, 50)])
def test_walker_groups_replay_the_job_and_match_the_oracle(window):
    """Production recorded per group of walkers (22 walkers in 5 ragged
    groups): the job ends exactly as after its own recorded sweeps (sums and
    every walker's state bit-identical to a twin job's), the groups' sums add
    up to the total, and each group's sums equal the oracle's for that walker
    range swept from the same state under the same weights."""
    L, T, nw, seed, groups, sweeps = 4, 2.0, 22, 17, 5, 300
    print(f"[analysis] walker groups window={window}", flush=True)
    a = MucaJob(L, T, nw, seed=seed, max_delta=1)
    b = MucaJob(L, T, nw, seed=seed, max_delta=1)
    for j in (a, b):
        if window is not None:
            j.set_window(*window)
        for _ in range(4):
            j.sweep(200)
            j.update_weights(j.reduce_hist())
    spins0, state0 = a.read_state()
    lnW = a.lnW
    assert lnW.tobytes() == b.lnW.tobytes()
    blocks, total = analysis.walker_blocks(a, groups, sweeps)
    b.reset_accum()
    b.sweep(sweeps, record=True)
    assert a.read_accum() == b.read_accum() == total
    sa, sta = a.read_state()
    sb, stb = b.read_state()
    assert np.array_equal(sa, sb) and np.array_equal(sta, stb)
    for k in ("H", "SJ", "SJJ", "SA", "SM2", "SM4"):
        assert [sum(col) for col in zip(*(blk[k] for blk in blocks))] == total[k]
    edges = [nw * g // groups for g in range(groups + 1)]
    for g in range(groups):
        x, y = edges[g], edges[g + 1]
        o = oracle.OracleJob(L, T, y - x, seed, lnW=lnW, first_walker=x)
        if window is not None:
            o.set_window(*window)
        assert o.lnW.tobytes() == lnW.tobytes()
        o.spins[:] = spins0[x:y]
        o.state[:] = state0[x:y]
        o.sweep(sweeps, record=True)
        assert o.bin_sums() == blocks[g], f"group {g}"
    with pytest.raises(ValueError):
        analysis.walker_blocks(a, nw + 1, 1)
    a.free()
    b.free()
