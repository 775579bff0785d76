"""ctypes binding of libmuca (include/muca.h): same names, argument marshalling only.

PyTorch supplies the device memory (uint8 tensors sized by muca_query_sizes)
and the HIP stream; every step of the method runs in libmuca's kernels and host
code.  The binding fails loudly when libmuca.so is missing: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmuca.so")

MUCA_OK = 0
MUCA_RECORD = 1
OBS_FIELDS = (
    "delta", "mean_EJ", "mean_ED", "mean_E", "mean_EJ2", "var_EJ", "var_ED",
    "C_field", "dC_dDelta", "cV", "mean_absM", "mean_M2", "mean_M4", "binder_U4",
    "edge_weight",
)
EXPORTS = (
    "muca_query_sizes", "muca_init", "muca_sweep", "muca_reduce_hist", "muca_update_weights",
    "muca_set_weights", "muca_get_weights", "muca_reweight", "muca_read_state", "muca_write_state",
    "muca_read_accum", "muca_reset_accum", "muca_set_stats", "muca_read_stats", "muca_set_launch", "muca_get_launch", "muca_host_tables",
    "muca_host_order", "muca_strerror", "muca_free", "muca_batch_query_size", "muca_batch_create",
    "muca_batch_set_launch", "muca_batch_get_launch", "muca_batch_sweep", "muca_batch_free", "muca_flatness", "muca_reweight_sums",
    "muca_reweight_hist", "muca_reweight_hist_sums", "muca_set_recursion", "muca_batch_sweep_static",
    "muca_set_window", "muca_get_window", "muca_host_walls", "muca_batch_submit", "muca_batch_poll",
    "muca_batch_finish", "muca_set_stream", "muca_get_recursion_state", "muca_set_recursion_state",
    "muca_write_accum",
)

# weight recursion flags (muca_set_recursion)
REC_ACCUMULATED = 1
REC_EXTRAPOLATE = 2


class MucaError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib().muca_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: error {code}: {msg}")


class muca_params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("T", ctypes.c_double), ("n_walkers", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("max_delta", ctypes.c_int32), ("first_walker", ctypes.c_int32)]


class muca_dev_buffers(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_void_p), ("walker_state", ctypes.c_void_p), ("hist", ctypes.c_void_p),
                ("tables", ctypes.c_void_p), ("accum", ctypes.c_void_p), ("obs", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libmuca.so (built by __graft_entry__.build()); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmuca.so not found at {LIB_PATH}: run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    P, vp, i32, i64, u32, dbl = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
    sz = P(ctypes.c_size_t)
    L.muca_query_sizes.argtypes = [P(muca_params), sz, sz, sz, sz, sz, sz]
    L.muca_init.argtypes = [P(muca_params), P(muca_dev_buffers), P(dbl), vp, P(vp)]
    L.muca_sweep.argtypes = [vp, i64, u32]
    L.muca_reduce_hist.argtypes = [vp, P(i64), i32]
    L.muca_update_weights.argtypes = [vp, P(i64), P(dbl), P(dbl)]
    L.muca_set_recursion.argtypes = [vp, ctypes.c_uint32]
    L.muca_set_weights.argtypes = [vp, P(dbl)]
    L.muca_get_weights.argtypes = [vp, P(dbl)]
    L.muca_reweight.argtypes = [vp, P(dbl), i32, P(dbl)]
    L.muca_read_state.argtypes = [vp, P(ctypes.c_int8), P(i64)]
    L.muca_write_state.argtypes = [vp, P(ctypes.c_int8), P(i64)]
    L.muca_read_accum.argtypes = [vp, P(i64), P(ctypes.c_uint64)]
    L.muca_reset_accum.argtypes = [vp]
    L.muca_set_stats.argtypes = [vp, i32]
    L.muca_read_stats.argtypes = [vp, P(i64), i32]
    L.muca_set_launch.argtypes = [vp, i32, i32, i32, i32]
    L.muca_get_launch.argtypes = [vp, P(i32), P(i32), P(i32), P(i32), P(i32)]
    L.muca_host_tables.argtypes = [i32, dbl, P(dbl), i32, i32, P(dbl), P(dbl), P(dbl)]
    L.muca_host_walls.argtypes = [i32, dbl, i32, i32, P(dbl)]
    L.muca_set_window.argtypes = [vp, i32, i32]
    L.muca_set_stream.argtypes = [vp, vp]
    L.muca_get_recursion_state.argtypes = [vp, P(dbl), P(ctypes.c_uint8)]
    L.muca_set_recursion_state.argtypes = [vp, P(dbl), P(ctypes.c_uint8)]
    L.muca_write_accum.argtypes = [vp, P(i64), P(ctypes.c_uint64)]
    L.muca_get_window.argtypes = [vp, P(i32), P(i32)]
    L.muca_host_order.argtypes = [i32, P(i32)]
    L.muca_strerror.argtypes = [ctypes.c_int]
    L.muca_strerror.restype = ctypes.c_char_p
    L.muca_free.argtypes = [vp]
    L.muca_free.restype = None
    L.muca_batch_query_size.argtypes = [P(vp), i32, sz]
    L.muca_batch_create.argtypes = [P(vp), i32, vp, ctypes.c_size_t, P(vp)]
    L.muca_batch_set_launch.argtypes = [vp, i32, i32, i32, i32]
    L.muca_batch_get_launch.argtypes = [vp, P(i32), P(i32), P(i32), P(i32)]
    L.muca_batch_sweep.argtypes = [vp, i64, u32]
    L.muca_batch_sweep_static.argtypes = [P(vp), i32, i64, u32]
    L.muca_batch_submit.argtypes = [vp, i64, u32]
    L.muca_batch_poll.argtypes = [vp, P(i32)]
    L.muca_batch_finish.argtypes = [vp]
    L.muca_batch_free.argtypes = [vp]
    L.muca_batch_free.restype = None
    L.muca_flatness.argtypes = [P(i64), i32, i32, P(dbl)]
    L.muca_reweight_sums.argtypes = [vp, P(i64), P(ctypes.c_uint64), P(dbl), i32, P(dbl)]
    L.muca_reweight_hist.argtypes = [vp, dbl, P(dbl)]
    L.muca_reweight_hist_sums.argtypes = [vp, P(i64), dbl, P(dbl)]
    for name in EXPORTS:
        if name not in ("muca_strerror", "muca_free", "muca_batch_free"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc != MUCA_OK:
        raise MucaError(rc, where)


def _p(a: np.ndarray, ct):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _params(L, T, n_walkers, seed, max_delta, first_walker=0) -> muca_params:
    return muca_params(int(L), float(T), int(n_walkers), int(seed) & 0xFFFFFFFFFFFFFFFF, int(max_delta),
                       int(first_walker))


def muca_query_sizes(L: int, T: float, n_walkers: int, seed: int = 0, max_delta: int = 0,
                     first_walker: int = 0) -> dict:
    s = [ctypes.c_size_t() for _ in range(6)]
    pr = _params(L, T, n_walkers, seed, max_delta, first_walker)
    _check(lib().muca_query_sizes(ctypes.byref(pr), *[ctypes.byref(x) for x in s]), "muca_query_sizes")
    return dict(zip(("lattice", "walker_state", "hist", "tables", "accum", "obs"), [x.value for x in s]))


def muca_host_tables(L: int, T: float, lnW: np.ndarray, window=None):
    V = L ** 3
    lo, hi = (0, V) if window is None else window
    lw = np.ascontiguousarray(lnW, dtype=np.float64)
    Bp, Rp, Rm = np.zeros(25), np.zeros(V + 1), np.zeros(V + 1)
    D = ctypes.c_double
    _check(lib().muca_host_tables(L, float(T), _p(lw, D), int(lo), int(hi), _p(Bp, D), _p(Rp, D), _p(Rm, D)),
           "muca_host_tables")
    return Bp, Rp, Rm


def muca_host_walls(L: int, T: float, lo: int, hi: int, lnW: np.ndarray) -> np.ndarray:
    """lnW with the bins outside [lo, hi] replaced by the window's walls."""
    lw = np.array(lnW, dtype=np.float64)
    _check(lib().muca_host_walls(L, float(T), int(lo), int(hi), _p(lw, ctypes.c_double)), "muca_host_walls")
    return lw


def muca_flatness(hist: np.ndarray, lo: int, hi: int) -> float:
    h = np.ascontiguousarray(hist, dtype=np.int64)
    assert 0 <= lo <= hi < len(h)
    out = ctypes.c_double()
    _check(lib().muca_flatness(_p(h, ctypes.c_int64), int(lo), int(hi), ctypes.byref(out)), "muca_flatness")
    return out.value


def muca_host_order(L: int) -> np.ndarray:
    o = np.zeros(L ** 3, dtype=np.int32)
    _check(lib().muca_host_order(L, _p(o, ctypes.c_int32)), "muca_host_order")
    return o


class MucaJob:
    """One multicanonical job (one (L, T), n_walkers walkers, one weight function).

    Device buffers are torch uint8 tensors on `device`; work is ordered on
    `stream` (a torch.cuda.Stream, default: the device's current stream)."""

    def __init__(self, L: int, T: float, n_walkers: int, seed: int = 0, lnW: Optional[Sequence[float]] = None,
                 max_delta: int = 256, device=None, stream=None, first_walker: int = 0):
        import torch

        self.L, self.V, self.T = int(L), int(L) ** 3, float(T)
        self.beta = 0.0 if math.isinf(self.T) else 1.0 / self.T
        self.n_walkers, self.seed, self.max_delta = int(n_walkers), int(seed), int(max_delta)
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        sizes = muca_query_sizes(L, T, n_walkers, seed, max_delta, first_walker)
        self.sizes = sizes
        self._tensors = {}
        ptrs = {}
        for name, nbytes in sizes.items():
            t = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-t.data_ptr()) % 256
            self._tensors[name] = t
            ptrs[name] = t.data_ptr() + off
        self.buffers = muca_dev_buffers(**ptrs)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.first_walker = int(first_walker)
        pr = _params(L, T, n_walkers, seed, max_delta, first_walker)
        lw = None
        if lnW is not None:
            lw = np.ascontiguousarray(lnW, dtype=np.float64)
            assert lw.shape == (self.V + 1,)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib().muca_init(ctypes.byref(pr), ctypes.byref(self.buffers),
                                 _p(lw, ctypes.c_double) if lw is not None else None,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle))
        _check(rc, "muca_init")
        self._h = handle
        self.recursion = 0

    # -- the hot path -----------------------------------------------------
    def sweep(self, n_sweeps: int, record: bool = False):
        _check(lib().muca_sweep(self._h, int(n_sweeps), MUCA_RECORD if record else 0), "muca_sweep")

    def reduce_hist(self, reset: bool = True) -> np.ndarray:
        h = np.zeros(self.V + 1, dtype=np.int64)
        _check(lib().muca_reduce_hist(self._h, _p(h, ctypes.c_int64), 1 if reset else 0), "muca_reduce_hist")
        return h

    def update_weights(self, hist: np.ndarray) -> float:
        h = np.ascontiguousarray(hist, dtype=np.int64)
        flat = ctypes.c_double()
        _check(lib().muca_update_weights(self._h, _p(h, ctypes.c_int64), None, ctypes.byref(flat)),
               "muca_update_weights")
        return flat.value

    def reweight(self, deltas) -> np.ndarray:
        d = np.ascontiguousarray(deltas, dtype=np.float64)
        out = np.zeros((len(d), len(OBS_FIELDS)))
        _check(lib().muca_reweight(self._h, _p(d, ctypes.c_double), len(d), _p(out, ctypes.c_double)),
               "muca_reweight")
        return out

    def reweight_sums(self, sums: dict, deltas) -> np.ndarray:
        """Reweight per-bin sums given as exact integers (the read_accum format)."""
        V1 = self.V + 1
        s5 = np.array([[int(v) for v in sums[k]] for k in ("H", "SJ", "SJJ", "SA", "SM2")], dtype=np.int64)
        m4 = [int(v) for v in sums["SM4"]]
        sm4 = np.array([[v & 0xFFFFFFFFFFFFFFFF for v in m4], [v >> 64 for v in m4]], dtype=np.uint64)
        assert s5.shape == (5, V1)
        d = np.ascontiguousarray(deltas, dtype=np.float64)
        out = np.zeros((len(d), len(OBS_FIELDS)))
        _check(lib().muca_reweight_sums(self._h, _p(s5, ctypes.c_int64), _p(sm4, ctypes.c_uint64),
                                        _p(d, ctypes.c_double), len(d), _p(out, ctypes.c_double)), "muca_reweight_sums")
        return out

    def reweight_hist(self, delta: float) -> np.ndarray:
        """ln P(E_Delta) at Delta from the production histogram."""
        out = np.zeros(self.V + 1)
        _check(lib().muca_reweight_hist(self._h, float(delta), _p(out, ctypes.c_double)), "muca_reweight_hist")
        return out

    def reweight_hist_sums(self, hist, delta: float) -> np.ndarray:
        """ln P(E_Delta) at Delta from a caller-supplied histogram (V+1 counts)."""
        h = np.ascontiguousarray(hist, dtype=np.int64)
        assert h.shape == (self.V + 1,)
        out = np.zeros(self.V + 1)
        _check(lib().muca_reweight_hist_sums(self._h, _p(h, ctypes.c_int64), float(delta), _p(out, ctypes.c_double)),
               "muca_reweight_hist_sums")
        return out

    # -- weights, state, accumulators ---------------------------------------
    @property
    def lnW(self) -> np.ndarray:
        w = np.zeros(self.V + 1)
        _check(lib().muca_get_weights(self._h, _p(w, ctypes.c_double)), "muca_get_weights")
        return w

    def set_recursion(self, flags: int):
        """Weight recursion of update_weights from now on (REC_ACCUMULATED,
        REC_EXTRAPOLATE or 0 for the plain recursion); resets its statistics."""
        _check(lib().muca_set_recursion(self._h, int(flags)), "muca_set_recursion")
        self.recursion = int(flags)

    def set_stream(self, stream):
        """Order the job's later work on stream (a torch.cuda.Stream)."""
        _check(lib().muca_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)), "muca_set_stream")
        self.stream = stream

    def submit(self, n_sweeps: int, record: bool = False):
        """muca_sweep, then mark its completion on the job's stream."""
        import torch

        self.sweep(n_sweeps, record)
        self._done = torch.cuda.Event()
        self._done.record(self.stream)

    def poll(self) -> bool:
        """True when everything submitted has finished (never blocks)."""
        ev = getattr(self, "_done", None)
        return ev is None or ev.query()

    def set_window(self, lo: int, hi: int):
        """Confine the walkers to E_Delta in [lo, hi] (muca_set_window)."""
        _check(lib().muca_set_window(self._h, int(lo), int(hi)), "muca_set_window")

    @property
    def window(self) -> tuple:
        lo, hi = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().muca_get_window(self._h, ctypes.byref(lo), ctypes.byref(hi)), "muca_get_window")
        return lo.value, hi.value

    def set_weights(self, lnW):
        w = np.ascontiguousarray(lnW, dtype=np.float64)
        assert w.shape == (self.V + 1,)
        _check(lib().muca_set_weights(self._h, _p(w, ctypes.c_double)), "muca_set_weights")

    def read_state(self):
        spins = np.zeros((self.n_walkers, self.V), dtype=np.int8)
        state = np.zeros((self.n_walkers, 4), dtype=np.int64)
        _check(lib().muca_read_state(self._h, _p(spins, ctypes.c_int8), _p(state, ctypes.c_int64)),
               "muca_read_state")
        return spins, state

    def write_state(self, spins: np.ndarray, state: np.ndarray):
        s = np.ascontiguousarray(spins, dtype=np.int8)
        st = np.ascontiguousarray(state, dtype=np.int64)
        _check(lib().muca_write_state(self._h, _p(s, ctypes.c_int8), _p(st, ctypes.c_int64)), "muca_write_state")

    def read_accum(self) -> dict:
        """Per-bin production sums as exact Python integers (same keys as the oracle)."""
        V1 = self.V + 1
        sums = np.zeros((5, V1), dtype=np.int64)
        sm4 = np.zeros((2, V1), dtype=np.uint64)
        _check(lib().muca_read_accum(self._h, _p(sums, ctypes.c_int64), _p(sm4, ctypes.c_uint64)),
               "muca_read_accum")
        return {"H": [int(v) for v in sums[0]], "SJ": [int(v) for v in sums[1]], "SJJ": [int(v) for v in sums[2]],
                "SA": [int(v) for v in sums[3]], "SM2": [int(v) for v in sums[4]],
                "SM4": [int(lo) + (int(hi) << 64) for lo, hi in zip(sm4[0], sm4[1])], "V": self.V}

    def reset_accum(self):
        _check(lib().muca_reset_accum(self._h), "muca_reset_accum")

    def write_accum(self, sums: dict):
        """Restore production sums given as exact integers (the read_accum format)."""
        V1 = self.V + 1
        s5 = np.array([[int(v) for v in sums[k]] for k in ("H", "SJ", "SJJ", "SA", "SM2")], dtype=np.int64)
        m4 = [int(v) for v in sums["SM4"]]
        sm4 = np.array([[v & 0xFFFFFFFFFFFFFFFF for v in m4], [v >> 64 for v in m4]], dtype=np.uint64)
        assert s5.shape == (5, V1)
        _check(lib().muca_write_accum(self._h, _p(s5, ctypes.c_int64), _p(sm4, ctypes.c_uint64)), "muca_write_accum")

    def recursion_state(self):
        """(kacc, seen) of the weight recursion, for an exact checkpoint."""
        kacc = np.zeros(self.V, dtype=np.float64)
        seen = np.zeros(self.V + 1, dtype=np.uint8)
        _check(lib().muca_get_recursion_state(self._h, _p(kacc, ctypes.c_double), _p(seen, ctypes.c_uint8)),
               "muca_get_recursion_state")
        return kacc, seen

    def set_recursion_state(self, kacc, seen):
        k = np.ascontiguousarray(kacc, dtype=np.float64)
        sn = np.ascontiguousarray(seen, dtype=np.uint8)
        assert k.shape == (self.V,) and sn.shape == (self.V + 1,)
        _check(lib().muca_set_recursion_state(self._h, _p(k, ctypes.c_double), _p(sn, ctypes.c_uint8)),
               "muca_set_recursion_state")

    def set_stats(self, enable: bool = True):
        _check(lib().muca_set_stats(self._h, 1 if enable else 0), "muca_set_stats")

    def read_stats(self, reset: bool = False) -> dict:
        v = np.zeros(3, dtype=np.int64)
        _check(lib().muca_read_stats(self._h, _p(v, ctypes.c_int64), 1 if reset else 0), "muca_read_stats")
        return {"passes": int(v[0]), "rounds": int(v[1]), "accepted": int(v[2])}

    def set_launch(self, waves_per_walker: int, blocks_per_lane: int, lds_tables: int = -1, packing: int = -1):
        _check(lib().muca_set_launch(self._h, waves_per_walker, blocks_per_lane, lds_tables, packing),
               "muca_set_launch")

    def get_launch(self) -> dict:
        v = [ctypes.c_int32() for _ in range(5)]
        _check(lib().muca_get_launch(self._h, *[ctypes.byref(x) for x in v]), "muca_get_launch")
        return dict(zip(("waves_per_walker", "blocks_per_lane", "lds_tables", "packed", "lds_bytes"),
                        [x.value for x in v]))

    def free(self):
        if getattr(self, "_h", None):
            lib().muca_free(self._h)
            self._h = None
            self._tensors = {}

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class MucaBatch:
    """Several MucaJobs (same device and stream) swept by one persistent launch."""

    def __init__(self, jobs: Sequence[MucaJob]):
        import torch

        self.jobs = list(jobs)
        arr = (ctypes.c_void_p * len(self.jobs))(*[j._h.value for j in self.jobs])
        nbytes = ctypes.c_size_t()
        _check(lib().muca_batch_query_size(arr, len(self.jobs), ctypes.byref(nbytes)), "muca_batch_query_size")
        dev = self.jobs[0].device
        self._buf = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        ptr = self._buf.data_ptr() + (-self._buf.data_ptr()) % 256
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            _check(lib().muca_batch_create(arr, len(self.jobs), ctypes.c_void_p(ptr), nbytes.value, ctypes.byref(h)),
                   "muca_batch_create")
        self._h = h

    def set_launch(self, waves_per_walker: int, blocks_per_lane: int, blocks: int = 0, packing: int = -1):
        _check(lib().muca_batch_set_launch(self._h, waves_per_walker, blocks_per_lane, blocks, packing),
               "muca_batch_set_launch")

    def get_launch(self) -> dict:
        """The shape in use: waves per walker of each job (in the order given),
        blocks per lane, packing, LDS bytes."""
        w = (ctypes.c_int32 * len(self.jobs))()
        b, pk, lds = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().muca_batch_get_launch(self._h, w, ctypes.byref(b), ctypes.byref(pk), ctypes.byref(lds)),
               "muca_batch_get_launch")
        return {"waves_per_walker": list(w), "blocks_per_lane": b.value, "packed": pk.value, "lds_bytes": lds.value}

    def sweep(self, n_sweeps: int, record: bool = False):
        _check(lib().muca_batch_sweep(self._h, int(n_sweeps), MUCA_RECORD if record else 0), "muca_batch_sweep")

    def submit(self, n_sweeps: int, record: bool = False):
        """Enqueue n_sweeps sweeps and mark their completion (muca_batch_submit)."""
        _check(lib().muca_batch_submit(self._h, int(n_sweeps), MUCA_RECORD if record else 0), "muca_batch_submit")

    def poll(self) -> bool:
        """True when everything submitted has finished (never blocks)."""
        d = ctypes.c_int32()
        _check(lib().muca_batch_poll(self._h, ctypes.byref(d)), "muca_batch_poll")
        return bool(d.value)

    def finish(self):
        _check(lib().muca_batch_finish(self._h), "muca_batch_finish")

    def free(self):
        if getattr(self, "_h", None):
            lib().muca_batch_free(self._h)
            self._h = None
            self._buf = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def batch_sweep_static(jobs: Sequence[MucaJob], n_sweeps: int, record: bool = False):
    """muca_batch_sweep_static: one batched sweep of the jobs (same device and
    stream) whose job table and work list sit in the library's static device
    array, for callers that cannot allocate."""
    arr = (ctypes.c_void_p * len(jobs))(*[j._h.value for j in jobs])
    _check(lib().muca_batch_sweep_static(arr, len(jobs), int(n_sweeps), MUCA_RECORD if record else 0),
           "muca_batch_sweep_static")
