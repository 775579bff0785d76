"""GPU path vs oracle, through the C ABI: trajectories (lattices, E_J, E_Delta,
M, sweep counters), per-iteration histograms and weights bit for bit, per-bin
production sums bit for bit, reweighted observables to 1e-12 relative to
their value or to their condition scale (obs_tolerance states the bound)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1502_07214_amd import MucaBatch, MucaJob, OBS_FIELDS
from paper_1502_07214_amd import workloads

pytestmark = pytest.mark.gpu

COL = {k: i for i, k in enumerate(OBS_FIELDS)}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def abs_moments(sums, lnW, beta, deltas):
    """E|dJ dD| and E|dJ| dD^2 at each Delta (dJ, dD: bin mean of E_J and E_Delta
    minus their reweighted means).  They measure the size of the terms that the
    central moments are summed from; used only to size tolerances."""
    H = np.array(sums["H"], dtype=float)
    b = H > 0
    E = np.arange(len(H), dtype=float)[b]
    h = H[b]
    mJ = np.array(sums["SJ"], dtype=float)[b] / h
    lw = np.asarray(lnW)[b]
    out = []
    for d in deltas:
        a = -(beta * d) * E - lw
        p = np.exp(a - a.max()) * h
        p /= p.sum()
        dJ = mJ - (p * mJ).sum()
        dD = E - (p * E).sum()
        out.append(((p * np.abs(dJ * dD)).sum(), (p * np.abs(dJ) * dD * dD).sum()))
    return np.array(out)


def obs_tolerance(ref: np.ndarray, beta: float, V: int, absm: np.ndarray) -> np.ndarray:
    """1e-12 relative to each observable's value, or to its condition scale
    where that is larger: the sum of the magnitudes of the terms the value is
    summed from (a signed sum that nearly cancels, such as a central moment
    near a zero crossing, carries rounding errors of order eps times that sum,
    whatever the summation order).  For C, dC/dDelta and cV the scale is the
    same central moment taken over absolute values: beta E|dJ dD|,
    beta^2 E|dJ| dD^2 and beta^2 (Var E_J + 2|Delta| E|dJ dD| + Delta^2 Var E_Delta) / V.
    The third moment dC/dDelta is also allowed 64 rounding units of its
    sensitivity to the means it is centred on (see below): where the
    reweighted distribution sits on a few bins at the edge of the sampled
    range, the bin means differ from each other by 1e-4 of the means
    themselves and that sensitivity exceeds the absolute-sum scale."""
    sJ2 = np.maximum(ref[:, COL["var_EJ"]], 0.0)
    sD2 = np.maximum(ref[:, COL["var_ED"]], 0.0)
    eJ = np.abs(ref[:, COL["mean_EJ"]])
    eD = np.abs(ref[:, COL["mean_ED"]])
    d = np.abs(ref[:, COL["delta"]])
    floor = np.ones_like(ref)
    floor[:, COL["mean_EJ"]] = 3.0 * V
    floor[:, COL["mean_ED"]] = V
    floor[:, COL["mean_E"]] = 3.0 * V + d * V
    floor[:, COL["mean_EJ2"]] = (3.0 * V) ** 2
    floor[:, COL["var_EJ"]] = sJ2 + eJ + 1.0
    floor[:, COL["var_ED"]] = sD2 + eD + 1.0
    floor[:, COL["C_field"]] = beta * (absm[:, 0] + 1.0)
    floor[:, COL["dC_dDelta"]] = beta * beta * (absm[:, 1] + 1.0)
    floor[:, COL["cV"]] = beta * beta * (sJ2 + 2.0 * d * absm[:, 0] + d * d * sD2 + 1.0) / V
    floor[:, COL["mean_absM"]] = V
    floor[:, COL["mean_M2"]] = V * V
    floor[:, COL["mean_M4"]] = float(V) ** 4
    # dC/dDelta is summed from (E_J - <E_J>)(E_Delta - <E_Delta>)^2, so a
    # rounding error d in <E_J> moves it by d Var(E_Delta) and one in <E_Delta>
    # by 2 d cov: 64 units of FP64 rounding of those means, times that lever.
    sens = np.zeros_like(ref)
    sens[:, COL["dC_dDelta"]] = beta * beta * (eJ * sD2 + 2.0 * eD * absm[:, 0])
    return np.maximum(1e-12 * np.maximum(np.abs(ref), floor), 64.0 * np.finfo(np.float64).eps * sens)


def report_obs_errors(gpu, ref, tol):
    """Print, per observable, the largest |gpu - oracle| / |oracle| and the
    largest share of the tolerance used."""
    parts = []
    for j, name in enumerate(OBS_FIELDS[1:], start=1):
        ok = np.isfinite(ref[:, j]) & np.isfinite(gpu[:, j])
        if not ok.any():
            continue
        diff = np.abs(gpu[ok, j] - ref[ok, j])
        rel = diff / np.maximum(np.abs(ref[ok, j]), 1e-300)
        parts.append(f"{name} {rel.max():.1e} ({(diff / np.maximum(tol[ok, j], 1e-300)).max():.2f} of tol)")
    say("[parity] max rel err: " + ", ".join(parts))


def assert_obs_close(gpu, ref, beta, V, absm):
    tol = obs_tolerance(ref, beta, V, absm)
    report_obs_errors(gpu, ref, tol)
    both_nan = np.isnan(gpu) & np.isnan(ref)
    bad = ~both_nan & ~(np.abs(gpu - ref) <= tol)
    if bad.any():
        k, j = np.argwhere(bad)[0]
        raise AssertionError(f"{OBS_FIELDS[j]} at delta={ref[k, 0]}: gpu {gpu[k, j]!r} oracle {ref[k, j]!r} "
                             f"tol {tol[k, j]!r}")
    # plain 1e-12 relative on the observables summed from same-sign terms
    for name in ("mean_ED", "mean_EJ2", "mean_absM", "mean_M2", "mean_M4"):
        j = COL[name]
        assert np.all(np.abs(gpu[:, j] - ref[:, j]) <= 1e-12 * np.abs(ref[:, j]) + 1e-300), name


def run_both(L, T, nw, seed, iterations, sweeps, production, deltas, launch=None, lnW=None, threads=0, window=None,
             recursion=0):
    say(f"[parity] L={L} T={T} walkers={nw} seed={seed} it={iterations}x{sweeps} prod={production} launch={launch} "
        f"window={window} recursion={recursion}")
    job = MucaJob(L, T, nw, seed=seed, lnW=lnW, max_delta=max(1, len(deltas)))
    if launch is not None:
        job.set_launch(*launch)
    o = oracle.OracleJob(L, T, nw, seed, lnW=lnW, n_threads=threads)
    if recursion:
        job.set_recursion(recursion)
        o.set_recursion(recursion)
    if window is not None:
        job.set_window(*window)
        o.set_window(*window)
        assert job.window == tuple(window)
        assert job.lnW.tobytes() == o.lnW.tobytes(), "walls differ"
    spins, state = job.read_state()
    assert np.array_equal(spins, o.spins), "initial lattices differ"
    assert np.array_equal(state, o.state), "initial energies differ"
    for it in range(iterations):
        job.sweep(sweeps)
        hg = job.reduce_hist(reset=True)
        fg = job.update_weights(hg)
        o.sweep(sweeps)
        ho = o.take_hist()
        fo = o.update_weights(ho)
        assert np.array_equal(hg, ho), f"histogram differs at iteration {it}"
        assert fg == fo
        assert job.lnW.tobytes() == o.lnW.tobytes(), f"weights differ at iteration {it}"
    if production:
        job.sweep(production, record=True)
        o.sweep(production, record=True)
        assert np.array_equal(job.reduce_hist(), o.take_hist())
        sg, so = job.read_accum(), o.bin_sums()
        for k in ("H", "SJ", "SJJ", "SA", "SM2", "SM4"):
            assert sg[k] == so[k], f"production sum {k} differs"
    spins, state = job.read_state()
    assert np.array_equal(spins, o.spins), "lattices differ"
    assert np.array_equal(state, o.state), "walker energies / sweep counters differ"
    out = None
    if production and len(deltas):
        g = job.reweight(deltas)
        r = o.reweight(deltas)
        assert_obs_close(g, r, o.beta, o.V, abs_moments(o.bin_sums(), o.lnW, o.beta, deltas))
        out = (g, r)
    job.free()
    return out


def test_full_l4_t2_w16():
    """L=4, T=2.0, 16 walkers, flat start, 10 iterations x 2000 sweeps, 2000
    production sweeps, 200 Delta values: the whole job, bit for bit."""
    w = workloads.workload("l4_t2_w16")
    run_both(w["L"], w["T"], w["n_walkers"], w["seed"], w["iterations"], w["sweeps"], w["production"],
             workloads.delta_grid(w["deltas"]))


def test_truncated_l12_t2_w256():
    """L=12, T=2.0, all 256 walkers, 2 iterations x 1000 sweeps + 500 production."""
    w = workloads.workload("l12_t2_w256", truncated=True)
    run_both(w["L"], w["T"], w["n_walkers"], w["seed"], w["iterations"], w["sweeps"], w["production"],
             workloads.delta_grid(w["deltas"]))


@pytest.mark.parametrize("name", ["l12_t2_w256", "l16_t1_w1024"])
def test_full_size_benchmark_job_sampled(name):
    """A job at full size and in the default launch shape (the benchmark's:
    L=12, 256 walkers, 30 x 10^4 sweeps, 10^4 production sweeps, 200 Delta;
    and L=16, T=1, 1024 walkers, 60 x 2 10^4 sweeps).  The oracle cannot
    replay all of it in seconds, so: walkers sampled across the job are
    replayed on the oracle through the last iteration, from the GPU's state
    and weights, and must end bit-identical; every walker's tracked E_J,
    E_Delta, M equals a recomputation from its spins; every merged histogram
    counts each sweep of each walker once and contains the sampled walkers'
    own entries; the reweighting of the GPU's full production sums matches
    the oracle's reweighting of the same sums."""
    w = workloads.workload(name)
    L, T, nw, S = w["L"], w["T"], w["n_walkers"], w["sweeps"]
    deltas = workloads.delta_grid(w["deltas"])
    say(f"[parity] full-size benchmark job L={L} T={T} walkers={nw} {w['iterations']}x{S} + {w['production']}")
    job = MucaJob(L, T, nw, seed=w["seed"], max_delta=len(deltas))
    for it in range(w["iterations"] - 1):
        job.sweep(S)
        h = job.reduce_hist(reset=True)
        assert h.sum() == nw * S and h.min() >= 0
        job.update_weights(h)
    spins0, state0 = job.read_state()
    lnW0 = job.lnW.copy()
    job.sweep(S)
    h = job.reduce_hist(reset=True)
    assert h.sum() == nw * S
    spins1, state1 = job.read_state()
    assert np.all(state1[:, 3] == w["iterations"] * S)
    for k in range(nw):
        assert oracle.energies(L, spins1[k]) == tuple(int(x) for x in state1[k, :3]), f"walker {k} energies"
    part = np.zeros_like(h)
    for k in (0, nw // 3 + 12, nw - 1):
        o = oracle.OracleJob(L, T, 1, w["seed"], lnW=lnW0, first_walker=k)
        o.spins[0] = spins0[k]
        o.state[0] = state0[k]
        o.sweep(S)
        assert np.array_equal(o.spins[0], spins1[k]), f"walker {k} lattice differs after the last iteration"
        assert np.array_equal(o.state[0], state1[k]), f"walker {k} state differs after the last iteration"
        part += o.take_hist()
    assert np.all(h - part >= 0), "the merged histogram lacks entries of a sampled walker"
    job.update_weights(h)
    job.sweep(w["production"], record=True)
    assert job.reduce_hist(reset=True).sum() == nw * w["production"]
    sums = job.read_accum()
    assert sum(sums["H"]) == nw * w["production"]
    g = job.reweight(deltas)
    r = oracle.reweight(L ** 3, oracle.beta_of(T), job.lnW, sums, deltas)
    assert_obs_close(g, r, oracle.beta_of(T), L ** 3, abs_moments(sums, job.lnW, oracle.beta_of(T), deltas))
    job.free()


def test_saturation_job_sampled():
    """The saturation job at full size in its launch shape (65 536 walkers at
    L=8, one wave each, thresholds read through the caches; 10 + 100 sweeps
    under flat weights): sampled walkers replayed on the oracle from their
    initial state end bit-identical, every walker's energies equal a
    recomputation, and the histogram counts every sweep of every walker."""
    s = workloads.SATURATION
    L, T, nw = s["L"], s["T"], s["n_walkers"]
    say(f"[parity] saturation job L={L} walkers={nw}")
    job = MucaJob(L, T, nw, seed=s["seed"], max_delta=1)
    job.sweep(10)
    job.sweep(s["sweeps"])
    h = job.reduce_hist(reset=True)
    assert h.sum() == nw * (10 + s["sweeps"])
    spins, state = job.read_state()
    assert np.all(state[:, 3] == 10 + s["sweeps"])
    for w in range(0, nw, 97):
        assert oracle.energies(L, spins[w]) == tuple(int(v) for v in state[w, :3]), f"walker {w}"
    for w in (0, 4097, 33333, nw - 1):
        o = oracle.OracleJob(L, T, 1, s["seed"], first_walker=w)
        o.sweep(10)
        o.sweep(s["sweeps"])
        assert np.array_equal(o.spins[0], spins[w]) and np.array_equal(o.state[0], state[w]), f"walker {w}"
    job.free()


@pytest.mark.parametrize("L,nw", [(12, 131072), (16, 262144)])
def test_saturation_grid_sampled(L, nw):
    """Saturation runs of the grid at full size in the library's launch shape
    (10 + 20 sweeps under flat weights at T = 2): sampled walkers, the first
    and last among them, replayed on the oracle end bit-identical; sampled
    walkers' energies equal a recomputation; the histogram counts every sweep
    of every walker."""
    s = workloads.SATURATION
    assert (L, nw) in workloads.SATURATION_GRID
    say(f"[parity] saturation grid L={L} walkers={nw}")
    job = MucaJob(L, s["T"], nw, seed=s["seed"], max_delta=1)
    job.sweep(10)
    job.sweep(20)
    h = job.reduce_hist(reset=True)
    assert h.sum() == nw * 30
    spins, state = job.read_state()
    assert np.all(state[:, 3] == 30)
    for w in range(0, nw, 4099):
        assert oracle.energies(L, spins[w]) == tuple(int(v) for v in state[w, :3]), f"walker {w}"
    for w in (0, 65537, nw - 1):
        o = oracle.OracleJob(L, s["T"], 1, s["seed"], first_walker=w)
        o.sweep(10)
        o.sweep(20)
        assert np.array_equal(o.spins[0], spins[w]) and np.array_equal(o.state[0], state[w]), f"walker {w}"
    job.free()


def test_truncated_l16_t1_w1024():
    """L=16, T=1.0, all 1024 walkers, 2 iterations x 100 sweeps + 100 production."""
    w = workloads.workload("l16_t1_w1024", truncated=True)
    run_both(w["L"], w["T"], w["n_walkers"], w["seed"], w["iterations"], w["sweeps"], w["production"],
             workloads.delta_grid(w["deltas"]))


@pytest.mark.parametrize("wpw", [1, 2, 4])
@pytest.mark.parametrize("bpl,packing", [(1, 0), (1, 1), (2, 0)])
@pytest.mark.parametrize("lds_tables", [0, 1])
def test_launch_shapes_agree(wpw, bpl, packing, lds_tables):
    """Every launch shape replays the same chain (L=6: classes of 108 sites span
    several lane groups at 1 wave per walker; 7 walkers leave ragged blocks),
    with lattices in LDS as bytes or as 2-bit codes."""
    run_both(6, 1.4182, 7, 11, 3, 60, 40, np.linspace(1.0, 3.5, 9), launch=(wpw, bpl, lds_tables, packing))


@pytest.mark.parametrize("L,wpw,lds_tables", [(5, 1, 1), (9, 2, 0), (12, 4, 1), (16, 1, 0), (24, 4, 0)])
def test_packed_lattices_agree(L, wpw, lds_tables):
    """Packed lattices (2-bit codes in LDS) replay the sequential chain at odd
    L (3-colour classes straddling 4-site blocks), with neighbour positions in
    registers (few passes per sweep) and read per pass (many), and at L=24."""
    run_both(L, 1.2, 6, 40 + L, 2, 12, 8, np.linspace(2.5, 3.2, 5), launch=(wpw, 1, lds_tables, 1))


@pytest.mark.parametrize("L", [2, 3, 5, 7, 9])
def test_small_and_odd_lattices(L):
    """L=2 (multiplicity-2 neighbours), odd L (3-colour order whose classes
    straddle 4-site blocks)."""
    run_both(L, 1.0 if L % 2 else 2.0, 5, 100 + L, 3, 40, 30, np.linspace(0.5, 3.5, 7))


def test_beta_zero_and_low_temperature():
    run_both(4, float("inf"), 4, 3, 2, 50, 20, np.array([0.0, 1.0]))
    run_both(4, 0.3, 4, 4, 2, 50, 20, np.array([2.5, 3.0, 3.5]))


def test_large_lattice_l32_global_tables():
    """L=32: V=32768, thresholds and neighbour table too large for LDS."""
    run_both(32, 2.0, 4, 5, 1, 4, 2, np.array([1.0, 2.5]))


def test_tilted_start_weights():
    L, T = 8, 1.0
    V = L ** 3
    lnW = np.array([-(2.9 / T) * E for E in range(V + 1)])
    run_both(L, T, 12, 6, 2, 30, 30, np.linspace(2.5, 3.3, 17), lnW=lnW)


def test_zero_sweeps_and_errors():
    job = MucaJob(4, 2.0, 3, seed=1, max_delta=2)
    s0, st0 = job.read_state()
    job.sweep(0)
    s1, st1 = job.read_state()
    assert np.array_equal(s0, s1) and np.array_equal(st0, st1)
    from paper_1502_07214_amd.muca import MucaError
    with pytest.raises(MucaError) as e:
        job.reweight([1.0])
    assert e.value.code == -4  # nothing recorded
    job.sweep(5, record=True)
    with pytest.raises(MucaError) as e:
        job.reweight([1.0, 2.0, 3.0])
    assert e.value.code == -3  # more than max_delta
    with pytest.raises(MucaError):
        job.sweep(-1)
    with pytest.raises(MucaError):
        job.set_launch(3, 1)
    job.free()


def test_checkpoint_resume_bit_exact():
    L, T, nw = 6, 1.4182, 8
    a = MucaJob(L, T, nw, seed=9, max_delta=4)
    a.sweep(30)
    a.update_weights(a.reduce_hist())
    spins, state = a.read_state()
    lnW = a.lnW
    a.sweep(40)
    ha = a.reduce_hist()
    sa, sta = a.read_state()
    b = MucaJob(L, T, nw, seed=9, max_delta=4)
    b.write_state(spins, state)
    b.set_weights(lnW)
    b.sweep(40)
    assert np.array_equal(b.reduce_hist(), ha)
    sb, stb = b.read_state()
    assert np.array_equal(sa, sb) and np.array_equal(sta, stb)
    a.free()
    b.free()


@pytest.mark.parametrize("batched", [False, True])
def test_walker_split_equals_whole(batched):
    """Sharding over walkers (one sub-job per device, say): sub-jobs holding
    walker ranges [first, first + n) of the same seed, each updating its
    weights with the sum of all sub-jobs' histograms (what an all-reduce
    gives), replay the whole job exactly: merged histograms, weights, and
    every walker's lattice and energies, over several iterations; the sub-jobs
    swept one by one or in one batched launch."""
    L, T, nw, seed = 7, 1.4182, 11, 12
    ranges = ((0, 3), (3, 5), (8, 1), (9, 2))
    say(f"[parity] walker split L={L} walkers={nw} ranges={ranges} batched={batched}")
    whole = MucaJob(L, T, nw, seed=seed, max_delta=1)
    subs = [MucaJob(L, T, n, seed=seed, max_delta=1, first_walker=f) for f, n in ranges]
    batch = MucaBatch(subs) if batched else None
    for it in range(4):
        whole.sweep(30)
        if batch is not None:
            batch.sweep(30)
        else:
            for j in subs:
                j.sweep(30)
        h = whole.reduce_hist()
        merged = sum(j.reduce_hist() for j in subs)
        assert np.array_equal(h, merged), f"iteration {it}"
        whole.update_weights(h)
        for j in subs:
            j.update_weights(merged)
            assert j.lnW.tobytes() == whole.lnW.tobytes()
    spins, state = whole.read_state()
    for (f, n), j in zip(ranges, subs):
        sp, st = j.read_state()
        assert np.array_equal(sp, spins[f:f + n]) and np.array_equal(st, state[f:f + n])
    if batch is not None:
        batch.free()
    for j in subs + [whole]:
        j.free()


def test_first_walker_against_oracle():
    """A sub-job's walkers are the oracle's walkers of the same global indices."""
    L, T, seed, f, n = 5, 2.0, 33, 1000, 4
    j = MucaJob(L, T, n, seed=seed, max_delta=1, first_walker=f)
    o = oracle.OracleJob(L, T, n, seed, first_walker=f)
    sp, st = j.read_state()
    assert np.array_equal(sp, o.spins) and np.array_equal(st, o.state)
    j.sweep(20)
    o.sweep(20)
    assert np.array_equal(j.reduce_hist(), o.take_hist())
    sp, st = j.read_state()
    assert np.array_equal(sp, o.spins) and np.array_equal(st, o.state)
    j.free()


def test_checkpoint_resume_accumulated_recursion_and_production():
    """An exact checkpoint under the accumulated + extrapolating recursion
    restores walkers, weights, the recursion's pair weights and visited bins,
    and the production sums recorded so far: the resumed job continues bit for
    bit like the original."""
    L, T, nw, seed = 6, 1.2, 8, 19
    a = MucaJob(L, T, nw, seed=seed, max_delta=4)
    a.set_recursion(3)
    for _ in range(3):
        a.sweep(40)
        a.update_weights(a.reduce_hist())
    a.sweep(30, record=True)
    a.reduce_hist()
    spins, state = a.read_state()
    lnW, (kacc, seen), sums = a.lnW, a.recursion_state(), a.read_accum()
    assert kacc.max() > 0 and seen.sum() > 0
    a.sweep(30, record=True)
    a.reduce_hist()
    final_sums = a.read_accum()
    for _ in range(2):
        a.sweep(40)
        a.update_weights(a.reduce_hist())
    b = MucaJob(L, T, nw, seed=seed, max_delta=4)
    b.set_recursion(3)
    b.write_state(spins, state)
    b.set_weights(lnW)
    b.set_recursion_state(kacc, seen)
    b.write_accum(sums)
    b.sweep(30, record=True)
    b.reduce_hist()
    assert b.read_accum() == final_sums
    for _ in range(2):
        b.sweep(40)
        b.update_weights(b.reduce_hist())
    assert a.lnW.tobytes() == b.lnW.tobytes()
    sa, sta = a.read_state()
    sb, stb = b.read_state()
    assert np.array_equal(sa, sb) and np.array_equal(sta, stb)
    ka, na = a.recursion_state()
    kb, nb = b.recursion_state()
    assert ka.tobytes() == kb.tobytes() and np.array_equal(na, nb)
    a.free()
    b.free()


@pytest.mark.parametrize("wpw", [1, 2, 4])
def test_jagged_weights_many_rounds(wpw):
    """Weights with strong bin-to-bin noise make decisions flip with every
    change of the guessed E_Delta: long cascades, many fixed-point rounds and,
    with several waves per walker, several exchanges per pass.  The chain must
    still be the sequential one."""
    L, T, nw, seed = 10, 1.5, 9, 41
    V = L ** 3
    rng = np.random.default_rng(5)
    lnW = -(2.8 / T) * np.arange(V + 1) + rng.normal(0.0, 1.5, size=V + 1)
    say(f"[parity] jagged weights L={L} walkers={nw} wpw={wpw}")
    job = MucaJob(L, T, nw, seed=seed, lnW=lnW, max_delta=1)
    job.set_launch(wpw, 1, -1)
    job.set_stats(True)
    o = oracle.OracleJob(L, T, nw, seed, lnW=lnW)
    job.sweep(40)
    o.sweep(40)
    st = job.read_stats()
    say(f"[parity] jagged weights: {st['rounds'] / st['passes']:.1f} rounds per pass (summed over waves)")
    assert np.array_equal(job.reduce_hist(), o.take_hist())
    spins, state = job.read_state()
    assert np.array_equal(spins, o.spins) and np.array_equal(state, o.state)
    # the case is a stress case: far more rounds than the 2 of smooth weights
    assert st["rounds"] / st["passes"] > 4 * wpw, st
    job.free()


@pytest.mark.parametrize("path", ["plain", "batched"])
def test_sum_of_m4_carries_past_64_bits(path):
    """The 128-bit per-bin sums of M^4 (carry detected on each 64-bit atomic)
    against the oracle's 128-bit sums: L = 30 lattices loaded fully ordered
    (M = V, M^4 = 5.3e17) at T = 0.5, where a few vacancies come and go, so
    nearly every sweep adds about V^4 to the bins near E_Delta = V and the
    sums pass 2^64 several times.  Run through the plain launch and through a
    batched launch next to a small job."""
    L, T, nw, sweeps, seed = 30, 0.5, 4, 48, 78
    V = L ** 3
    say(f"[parity] sum of M^4 past 2^64: L={L} T={T} walkers={nw} sweeps={sweeps} path={path}")
    job = MucaJob(L, T, nw, seed=seed, max_delta=2)
    job.write_state(np.ones((nw, V), dtype=np.int8), np.tile(np.array([-3 * V, V, V, 0], dtype=np.int64), (nw, 1)))
    o = oracle.OracleJob(L, T, nw, seed)
    o.spins[:] = 1
    o.state[:] = [-3 * V, V, V, 0]
    if path == "batched":
        other = MucaJob(4, 2.0, 8, seed=5, max_delta=1)
        batch = MucaBatch([job, other])
        batch.sweep(sweeps, record=True)
        batch.free()
        other.free()
    else:
        job.sweep(sweeps, record=True)
    o.sweep(sweeps, record=True)
    assert np.array_equal(job.reduce_hist(), o.take_hist())
    sg, so = job.read_accum(), o.bin_sums()
    for k in ("H", "SJ", "SJJ", "SA", "SM2", "SM4"):
        assert sg[k] == so[k], f"production sum {k} differs"
    assert max(v >> 64 for v in sg["SM4"]) >= 2, "the case must carry past 2^64"
    spins, state = job.read_state()
    assert np.array_equal(spins, o.spins) and np.array_equal(state, o.state)
    r = o.reweight([2.0, 3.0])
    g = job.reweight([2.0, 3.0])
    assert np.all(np.abs(g[:, COL["mean_M4"]] - r[:, COL["mean_M4"]]) <= 1e-12 * np.abs(r[:, COL["mean_M4"]]))
    job.free()


@pytest.mark.parametrize("recursion", [0, 3])
def test_window_job_bit_exact(recursion):
    """A job confined to an E_Delta window that holds its walkers' start (L=8,
    T=1, start tilted to Delta* = 2.944, window [200, 420] of V = 512): every
    histogram, weight array (walls included), lattice and production sum bit
    for bit, for the plain and the accumulated + extrapolating recursion."""
    L, T = 8, 1.0
    lnW = -(2.944 / T) * np.arange(L ** 3 + 1)
    run_both(L, T, 32, 17, 4, 200, 200, np.linspace(2.8, 3.1, 31), lnW=lnW, window=(200, 420),
             recursion=recursion)


@pytest.mark.parametrize("launch", [(1, 1, -1), (4, 1, 1), (2, 2, 0)])
def test_window_entered_from_outside(launch):
    """Random lattices sit near E_Delta = 2V/3 = 667, above the window [100, 400]
    of L=10, T=2: the walls take the walkers in and the tables keep them there
    (odd and even launch shapes); entries before they arrive fall outside the
    window and are not used."""
    run_both(10, 2.0, 12, 23, 3, 150, 100, np.linspace(2.3, 2.8, 11), window=(100, 400), launch=launch)


def test_window_batched_equals_oracle():
    """Windowed jobs in one batched launch: each equals its oracle replay."""
    specs = [(8, 1.0, 16, 31, (150, 480)), (6, 2.0, 9, 32, (20, 120)), (12, 0.9, 8, 33, (400, 1700))]
    jobs, ors = [], []
    for L, T, n, seed, win in specs:
        lnW = -(2.9 / T) * np.arange(L ** 3 + 1)
        j = MucaJob(L, T, n, seed=seed, lnW=lnW, max_delta=1)
        j.set_window(*win)
        o = oracle.OracleJob(L, T, n, seed, lnW=lnW)
        o.set_window(*win)
        jobs.append(j)
        ors.append(o)
    say("[parity] windowed batch of 3 jobs")
    batch = MucaBatch(jobs)
    for it in range(3):
        batch.sweep(60, record=(it == 2))
        for j, o in zip(jobs, ors):
            o.sweep(60, record=(it == 2))
            hg, ho = j.reduce_hist(), o.take_hist()
            assert np.array_equal(hg, ho)
            if it < 2:
                assert j.update_weights(hg) == o.update_weights(ho)
                assert j.lnW.tobytes() == o.lnW.tobytes()
    batch.free()
    for j, o in zip(jobs, ors):
        sg, so = j.read_accum(), o.bin_sums()
        assert all(sg[k] == so[k] for k in ("H", "SJ", "SJJ", "SA", "SM2", "SM4"))
        spins, state = j.read_state()
        assert np.array_equal(spins, o.spins) and np.array_equal(state, o.state)
        j.free()
