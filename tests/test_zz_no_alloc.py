"""The batched sweep that allocates nothing (muca_batch_sweep_static: job table,
work list and counter in the library's static device array) against the
batched sweep with a caller-provided buffer (muca_batch_create +
muca_batch_sweep) on clones of the same jobs: histograms, production sums,
lattices and walker state bit-identical, on two calls in a row, the second
with fewer jobs and walkers than the first."""
import sys

import numpy as np
import pytest

from paper_1502_07214_amd import MucaBatch, MucaJob
from paper_1502_07214_amd.muca import MucaError, batch_sweep_static

pytestmark = pytest.mark.gpu


def _make(specs):
    return [MucaJob(L, T, n, seed=s, max_delta=1) for (L, T, n, s) in specs]


def _assert_same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x.reduce_hist(), y.reduce_hist()), f"histogram of L={x.L} T={x.T}"
        assert x.read_accum() == y.read_accum(), f"production sums of L={x.L} T={x.T}"
        sx, tx = x.read_state()
        sy, ty = y.read_state()
        assert np.array_equal(sx, sy) and np.array_equal(tx, ty), f"walkers of L={x.L} T={x.T}"


def test_static_batch_equals_buffered_batch():
    first = [(8, 0.9, 64, 1), (12, 2.0, 40, 2), (5, 1.4182, 9, 3), (16, 1.0, 8, 4), (20, 2.0, 4, 9)]
    second = [(6, 2.0, 5, 7), (10, 1.0, 33, 8)]
    for call, (specs, sweeps) in enumerate(((first, 30), (second, 17))):
        print(f"[no-alloc] call {call}: {len(specs)} jobs, {sum(s[2] for s in specs)} walkers, "
              f"{sweeps} sweeps", flush=True)
        sys.stdout.flush()
        a, b = _make(specs), _make(specs)
        batch_sweep_static(a, sweeps, record=True)
        batch_sweep_static(a, 3)
        mb = MucaBatch(b)
        mb.sweep(sweeps, record=True)
        mb.sweep(3)
        mb.free()
        _assert_same(a, b)
        for j in a + b:
            j.free()


def test_static_batch_limits():
    jobs = _make([(4, 2.0, 2, 1), (4, 2.0, 2, 2)])
    with pytest.raises(MucaError) as e:
        batch_sweep_static([jobs[0], jobs[0]], 1)
    assert e.value.code == -1  # the same job twice
    with pytest.raises(MucaError) as e:
        batch_sweep_static(jobs, -1)
    assert e.value.code == -1
    # one wave per walker: tiles of 4 walkers, 65536 tiles at most
    big = MucaJob(2, 2.0, 4 * 65536 + 1, seed=3, max_delta=1)
    with pytest.raises(MucaError) as e:
        batch_sweep_static([big], 1)
    assert e.value.code == -3  # more tiles than the static work list holds
    batch_sweep_static(jobs, 0)
    for j in jobs + [big]:
        j.free()
