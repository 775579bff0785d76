"""Batched persistent launch: every job swept inside a batch equals the same
job swept alone (lattices, energies, histograms, weights, production sums),
and the oracle, for mixed L (even and odd) and T."""
import numpy as np
import pytest

import oracle
from paper_1502_07214_amd import MucaBatch, MucaJob

pytestmark = pytest.mark.gpu

MIX = [(8, 0.9, 7, 11), (5, 2.0, 12, 12), (10, 1.4182, 5, 13), (4, 1.0, 9, 14), (7, 2.0, 3, 15)]


def iterate(jobs, sweep, iterations, sweeps):
    hists = []
    for it in range(iterations):
        sweep(sweeps)
        hs = [j.reduce_hist() for j in jobs]
        for j, h in zip(jobs, hs):
            j.update_weights(h)
        hists.append(hs)
    return hists


@pytest.mark.parametrize("shape", [(0, 1, 0, 0), (0, 2), (1, 1, 0, 0), (1, 2), (2, 1, 0, 0), (4, 1, 0, 0), (4, 2),
                                   (0, 1, 0, 1), (1, 1, 0, 1), (2, 1, 0, 1), (4, 1, 0, 1)])
def test_batch_equals_plain(shape):
    print(f"[batch] mixed jobs {MIX} shape {shape}", flush=True)
    a = [MucaJob(L, T, nw, seed=s, max_delta=4) for (L, T, nw, s) in MIX]
    b = [MucaJob(L, T, nw, seed=s, max_delta=4) for (L, T, nw, s) in MIX]
    batch = MucaBatch(a)
    batch.set_launch(*shape)
    ha = iterate(a, batch.sweep, 3, 40)
    hb = iterate(b, lambda n: [j.sweep(n) for j in b], 3, 40)
    for it in range(3):
        for x, y in zip(ha[it], hb[it]):
            assert np.array_equal(x, y)
    batch.sweep(30, record=True)
    for j in b:
        j.sweep(30, record=True)
    for ja, jb in zip(a, b):
        sa, sta = ja.read_state()
        sb, stb = jb.read_state()
        assert np.array_equal(sa, sb) and np.array_equal(sta, stb)
        assert ja.lnW.tobytes() == jb.lnW.tobytes()
        assert ja.read_accum() == jb.read_accum()
        assert np.array_equal(ja.reweight([1.0, 2.5, 3.0]), jb.reweight([1.0, 2.5, 3.0]))
    batch.free()
    for j in a + b:
        j.free()


def test_batch_matches_oracle():
    jobs = [MucaJob(L, T, nw, seed=s, max_delta=2) for (L, T, nw, s) in MIX[:3]]
    batch = MucaBatch(jobs)
    orcs = [oracle.OracleJob(L, T, nw, s) for (L, T, nw, s) in MIX[:3]]
    for it in range(2):
        batch.sweep(25)
        for j, o in zip(jobs, orcs):
            h = j.reduce_hist()
            j.update_weights(h)
            o.sweep(25)
            ho = o.take_hist()
            o.update_weights(ho)
            assert np.array_equal(h, ho)
    for j, o in zip(jobs, orcs):
        s, st = j.read_state()
        assert np.array_equal(s, o.spins) and np.array_equal(st, o.state)
    batch.free()


def test_batch_rejects_bad_input():
    from paper_1502_07214_amd.muca import MucaError
    j = MucaJob(4, 2.0, 2, seed=0, max_delta=1)
    with pytest.raises(MucaError):
        MucaBatch([j, j])
    batch = MucaBatch([j])
    with pytest.raises(MucaError):
        batch.set_launch(3, 1)
    with pytest.raises(MucaError):
        batch.sweep(-1)
    batch.free()
    j.free()


@pytest.mark.parametrize("shape", [(1, 1), (4, 1)])
def test_batch_mixes_staged_and_cached_tables(shape):
    """A large lattice fills the batch's LDS with spins, so only the smallest
    jobs get their tables staged in LDS; the others read them through the
    caches in the same launch."""
    mix = [(20, 1.5, 2, 21), (4, 1.0, 9, 14), (5, 2.0, 6, 12), (8, 0.9, 3, 11)]
    print(f"[batch] staged + cached tables {mix} shape {shape}", flush=True)
    a = [MucaJob(L, T, nw, seed=s, max_delta=1) for (L, T, nw, s) in mix]
    b = [MucaJob(L, T, nw, seed=s, max_delta=1) for (L, T, nw, s) in mix]
    batch = MucaBatch(a)
    batch.set_launch(*shape)
    ha = iterate(a, batch.sweep, 2, 20)
    hb = iterate(b, lambda n: [j.sweep(n) for j in b], 2, 20)
    for it in range(2):
        for x, y in zip(ha[it], hb[it]):
            assert np.array_equal(x, y)
    for ja, jb in zip(a, b):
        sa, sta = ja.read_state()
        sb, stb = jb.read_state()
        assert np.array_equal(sa, sb) and np.array_equal(sta, stb)
        assert ja.lnW.tobytes() == jb.lnW.tobytes()
    batch.free()
    for j in a + b:
        j.free()


# Large lattices with few walkers next to small ones: the per-job launch
# shape (waves per walker 0) gives the L=16 and L=14 walkers four waves each
# and the small jobs one, in the same launch.
PER_JOB_MIX = [(16, 2.0, 5, 31), (4, 1.0, 9, 14), (14, 1.0, 3, 32), (5, 2.0, 6, 12), (8, 0.9, 7, 11), (7, 1.4182, 4, 15)]


@pytest.mark.parametrize("bpl", [1, 2])
def test_batch_per_job_waves_per_walker(bpl):
    print(f"[batch] per-job waves per walker {PER_JOB_MIX} bpl {bpl}", flush=True)
    a = [MucaJob(L, T, nw, seed=s, max_delta=3) for (L, T, nw, s) in PER_JOB_MIX]
    b = [MucaJob(L, T, nw, seed=s, max_delta=3) for (L, T, nw, s) in PER_JOB_MIX]
    batch = MucaBatch(a)
    assert batch.get_launch()["waves_per_walker"] == [1] * len(PER_JOB_MIX)
    batch.set_launch(0, bpl)
    shape = batch.get_launch()
    assert shape["waves_per_walker"] == [4, 1, 4, 1, 1, 1] and shape["blocks_per_lane"] == bpl
    ha = iterate(a, batch.sweep, 3, 30)
    hb = iterate(b, lambda n: [j.sweep(n) for j in b], 3, 30)
    for it in range(3):
        for x, y in zip(ha[it], hb[it]):
            assert np.array_equal(x, y)
    batch.sweep(20, record=True)
    for j in b:
        j.sweep(20, record=True)
    for ja, jb in zip(a, b):
        sa, sta = ja.read_state()
        sb, stb = jb.read_state()
        assert np.array_equal(sa, sb) and np.array_equal(sta, stb)
        assert ja.lnW.tobytes() == jb.lnW.tobytes()
        assert ja.read_accum() == jb.read_accum()
    batch.free()
    for j in a + b:
        j.free()


def test_batch_per_job_matches_oracle():
    mix = [(14, 1.0, 2, 41), (4, 2.0, 5, 42), (6, 1.0, 3, 43)]
    print(f"[batch] per-job waves per walker vs oracle {mix}", flush=True)
    jobs = [MucaJob(L, T, nw, seed=s, max_delta=1) for (L, T, nw, s) in mix]
    batch = MucaBatch(jobs)
    batch.set_launch(0, 1)
    assert batch.get_launch()["waves_per_walker"] == [4, 1, 1]
    orcs = [oracle.OracleJob(L, T, nw, s) for (L, T, nw, s) in mix]
    for it in range(2):
        batch.sweep(6)
        for j, o in zip(jobs, orcs):
            h = j.reduce_hist()
            j.update_weights(h)
            o.sweep(6)
            ho = o.take_hist()
            o.update_weights(ho)
            assert np.array_equal(h, ho)
    for j, o in zip(jobs, orcs):
        s, st = j.read_state()
        assert np.array_equal(s, o.spins) and np.array_equal(st, o.state)
    batch.free()
    for j in jobs:
        j.free()


def test_full_size_batched_workload_sampled():
    """The batched workload at full size (19 jobs of mixed L and T, 4096
    walkers, 10 iterations x 1000 sweeps, one persistent launch per iteration
    in the default shape): in every job the histograms count each sweep of
    each walker once and every walker's tracked E_J, E_Delta, M equals a
    recomputation from its spins; the first and the last walker of the largest
    and the smallest lattice's jobs, and of one in between, are replayed on the
    oracle through the last iteration from the GPU's state and weights and end
    bit-identical, their entries contained in the merged histogram."""
    from paper_1502_07214_amd import workloads
    specs = workloads.batched_jobs()
    it, sw = workloads.BATCHED["iterations"], workloads.BATCHED["sweeps"]
    print(f"[batch] full-size batched workload: {len(specs)} jobs, {sum(n for _, _, n, _ in specs)} walkers, {it}x{sw}",
          flush=True)
    jobs = [MucaJob(L, T, n, seed=s, max_delta=1) for (L, T, n, s) in specs]
    batch = MucaBatch(jobs)
    for k in range(it - 1):
        batch.sweep(sw)
        for j, (L, T, n, s) in zip(jobs, specs):
            h = j.reduce_hist(reset=True)
            assert h.sum() == n * sw
            j.update_weights(h)
    before = [(j.read_state(), j.lnW.copy()) for j in jobs]
    batch.sweep(sw)
    picks = sorted(range(len(specs)), key=lambda x: specs[x][0])
    picks = [picks[0], picks[len(picks) // 2], picks[-1]]
    for x, (j, (L, T, n, s)) in enumerate(zip(jobs, specs)):
        h = j.reduce_hist(reset=True)
        assert h.sum() == n * sw
        spins, state = j.read_state()
        assert np.all(state[:, 3] == it * sw)
        for w in range(n):
            assert oracle.energies(L, spins[w]) == tuple(int(v) for v in state[w, :3]), f"job {x} walker {w}"
        if x not in picks:
            continue
        (spins0, state0), lnW0 = before[x]
        part = np.zeros_like(h)
        for w in (0, n - 1):
            o = oracle.OracleJob(L, T, 1, s, lnW=lnW0, first_walker=w)
            o.spins[0] = spins0[w]
            o.state[0] = state0[w]
            o.sweep(sw)
            assert np.array_equal(o.spins[0], spins[w]) and np.array_equal(o.state[0], state[w]), \
                f"job (L={L}, T={T}) walker {w} differs after the last iteration"
            part += o.take_hist()
        assert np.all(h - part >= 0)
    batch.free()
    for j in jobs:
        j.free()


def test_tuned_shapes_keep_the_chain(tmp_path):
    """The autotuner's choices (timed on clones, written to a cache and read
    back from it) change speed only: the job and the batch swept in the tuned
    shapes equal the default shapes bit for bit."""
    from paper_1502_07214_amd import autotune

    cache = str(tmp_path / "tune.json")
    L, T, nw, seed = 10, 1.3, 24, 5
    shape = autotune.tune_job(L, T, nw, seed=seed, probe_sweeps=20, cache=cache)
    assert autotune.tune_job(L, T, nw, seed=seed, probe_sweeps=20, cache=cache) == shape
    a, b = MucaJob(L, T, nw, seed=seed, max_delta=1), MucaJob(L, T, nw, seed=seed, max_delta=1)
    a.set_launch(*shape)
    a.sweep(50)
    b.sweep(50)
    assert np.array_equal(a.reduce_hist(), b.reduce_hist())
    assert np.array_equal(a.read_state()[0], b.read_state()[0])
    specs = [(8, 1.0, 16, 1), (12, 2.0, 8, 2), (6, 0.9, 12, 3)]
    bshape = autotune.tune_batch(specs, probe_sweeps=10, cache=cache)
    # with finalists re-timed: a shape of the first pass, kept under its own key
    fshape = autotune.tune_batch(specs, probe_sweeps=10, cache=cache, finalists=3, repeats=2)
    entries = autotune._load(cache)
    fkey = [k for k in entries if k.startswith("batch4|") and k.endswith("|final3x2")]
    assert len(fkey) == 1 and list(fshape) == entries[fkey[0]]["shape"]
    assert set(entries[fkey[0]]["finalists"]) <= set(entries[fkey[0]]["timings"])
    assert str(tuple(fshape)) in entries[fkey[0]]["finalists"]
    ja = [MucaJob(L, T, n, seed=s, max_delta=1) for (L, T, n, s) in specs]
    jb = [MucaJob(L, T, n, seed=s, max_delta=1) for (L, T, n, s) in specs]
    ba, bb = MucaBatch(ja), MucaBatch(jb)
    ba.set_launch(*bshape)
    ba.sweep(30)
    bb.sweep(30)
    for x, y in zip(ja, jb):
        assert np.array_equal(x.reduce_hist(), y.reduce_hist())
        assert np.array_equal(x.read_state()[0], y.read_state()[0])
    for o in [a, b, ba, bb] + ja + jb:
        o.free()
    with pytest.raises(ValueError):
        autotune.tune_job(L, T, nw, seed=seed, probe_sweeps=5, shapes=[(3, 1, 0)])
