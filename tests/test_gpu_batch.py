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


@pytest.mark.parametrize("shape", [(1, 1), (1, 2), (2, 1), (4, 1), (4, 2)])
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
