"""Host-side checks of libmuca that need no GPU: the library loads and exports
every function include/muca.h declares; its threshold tables and visiting order
are bitwise identical to the oracle's (independent code, same host libm); its
argument checks return the documented error codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1502_07214_amd import muca

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "muca.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int|void)\s*\*?\s*(muca_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert "muca_sweep" in names and "muca_reweight" in names and len(names) >= 15
    lib = muca.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(muca.EXPORTS)


@pytest.mark.parametrize("L,T", [(2, 0.5), (4, 2.0), (12, 2.0), (16, 1.0), (5, 1.4182), (3, float("inf"))])
def test_host_tables_bitwise_equal_oracle(L, T):
    V = L ** 3
    rng = np.random.default_rng(L)
    for lnW in (np.zeros(V + 1), np.cumsum(rng.normal(0, 2.0, V + 1)), rng.normal(0, 800.0, V + 1)):
        a = muca.muca_host_tables(L, T, lnW)
        b = oracle.tables(V, oracle.beta_of(T), lnW)
        for x, y in zip(a, b):
            assert x.tobytes() == y.tobytes()


@pytest.mark.parametrize("L,T,lo,hi", [(2, 0.5, 2, 6), (4, 2.0, 10, 40), (12, 0.9, 300, 1500), (5, float("inf"), 0, 20),
                                        (6, 1.4182, 100, 216)])
def test_window_tables_and_walls_bitwise_equal_oracle(L, T, lo, hi):
    """The window's thresholds and walls equal the oracle's bit for bit."""
    V = L ** 3
    lnW = np.cumsum(np.random.default_rng(L + lo).normal(0, 2.0, V + 1))
    a = muca.muca_host_walls(L, T, lo, hi, lnW)
    job = oracle.OracleJob(L, T, 1, 0, lnW=lnW)
    job.set_window(lo, hi)
    assert a.tobytes() == job.lnW.tobytes()
    t = muca.muca_host_tables(L, T, a, window=(lo, hi))
    u = oracle.tables_window(V, oracle.beta_of(T), a, lo, hi)
    for x, y in zip(t, u):
        assert x.tobytes() == y.tobytes()


@pytest.mark.parametrize("L", range(2, 13))
def test_host_order_equals_oracle(L):
    assert np.array_equal(muca.muca_host_order(L), oracle.order(L))


def test_query_sizes():
    s = muca.muca_query_sizes(12, 2.0, 256, 0, 200)
    assert all(v > 0 and v % 256 == 0 for v in s.values())
    assert s["lattice"] >= 256 * 1728 and s["hist"] >= 8 * 1729 and s["accum"] >= 7 * 8 * 1729
    assert s["obs"] >= 200 * 16 * 8


@pytest.mark.parametrize("args", [
    (1, 2.0, 4, 0, 0), (33, 2.0, 4, 0, 0), (4, 0.0, 4, 0, 0), (4, -1.0, 4, 0, 0),
    (4, float("nan"), 4, 0, 0), (4, 2.0, 0, 0, 0), (4, 2.0, -3, 0, 0), (4, 2.0, 4, 0, -1),
    (4, 2.0, 4, 0, 70000), (4, 2.0, 4, 0, 0, -1), (4, 2.0, 4, 0, 0, 2 ** 31 - 2),
])
def test_invalid_params_rejected(args):
    with pytest.raises(muca.MucaError) as e:
        muca.muca_query_sizes(*args)
    assert e.value.code == -1


def test_init_argument_checks_without_device():
    lib = muca.lib()
    pr = muca.muca_params(4, 2.0, 4, 0, 8, 0)
    h = ctypes.c_void_p()
    bufs = muca.muca_dev_buffers(None, None, None, None, None, None)
    assert lib.muca_init(ctypes.byref(pr), ctypes.byref(bufs), None, None, ctypes.byref(h)) == -1
    bufs = muca.muca_dev_buffers(*([256 * 3 + 8] * 6))  # misaligned
    assert lib.muca_init(ctypes.byref(pr), ctypes.byref(bufs), None, None, ctypes.byref(h)) == -1
    assert lib.muca_init(ctypes.byref(pr), None, None, None, ctypes.byref(h)) == -1
    assert lib.muca_init(ctypes.byref(pr), ctypes.byref(bufs), None, None, None) == -1
    # calls on a null job
    assert lib.muca_sweep(None, 1, 0) == -1
    assert lib.muca_reduce_hist(None, None, 0) == -1
    assert lib.muca_update_weights(None, None, None, None) == -1
    assert lib.muca_reweight(None, None, 1, None) == -1
    assert lib.muca_batch_get_launch(None, None, None, None, None) == -1
    assert lib.muca_batch_set_launch(None, 1, 1, 0, -1) == -1
    assert lib.muca_batch_poll(None, None) == -1 and lib.muca_batch_finish(None) == -1
    assert lib.muca_set_window(None, 0, 1) == -1 and lib.muca_set_stream(None, None) == -1
    assert lib.muca_batch_sweep(None, 1, 0) == -1
    lib.muca_free(None)
    lib.muca_batch_free(None)


def test_strerror():
    lib = muca.lib()
    for code in range(0, -7, -1):
        assert lib.muca_strerror(code)
    assert b"invalid" in lib.muca_strerror(-1)
    assert lib.muca_strerror(-99) == b"unknown error code"
