"""Oracle for parallel multicanonical (MUCA) sampling of the 3D Blume-Capel model.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product library
never does, and the two share no code.

Paper: Zierenberg, Fytas and Janke, "Parallel multicanonical study of the
three-dimensional Blume-Capel model".  Sec. I, Eq. (1) defines the model and the
split H = E_J + Delta E_Delta; Sec. II defines the multicanonical weights
W(E_Delta) at fixed beta, the parallel iteration of the weights, time-series
reweighting to any Delta and the field derivative Eq. (FieldDerivative) with
its specific-heat-like special case Eq. (sph).

The sampling part (Philox generator, lattice, sweep, thresholds, recursion) is
plain C in ``muca_oracle.c``, called through ctypes; the reweighting is plain
numpy in float64 below, with the within-bin sums kept as exact Python integers.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, List, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "muca_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OBS_FIELDS = (
    "delta", "mean_EJ", "mean_ED", "mean_E", "mean_EJ2", "var_EJ", "var_ED",
    "C_field", "dC_dDelta", "cV", "mean_absM", "mean_M2", "mean_M4", "binder_U4",
    "edge_weight",
)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-pthread", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        u32p, i64p, u64p, dp = P(ctypes.c_uint32), P(ctypes.c_int64), P(ctypes.c_uint64), P(ctypes.c_double)
        i8p, i32p = P(ctypes.c_int8), P(ctypes.c_int32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_num_colours.argtypes = [ctypes.c_int]
        L.orc_num_colours.restype = ctypes.c_int
        L.orc_order.argtypes = [ctypes.c_int, i32p]
        L.orc_order.restype = None
        L.orc_energies.argtypes = [ctypes.c_int, i8p, i64p]
        L.orc_energies.restype = None
        L.orc_init_walker.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, i8p]
        L.orc_init_walker.restype = None
        L.orc_init.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, i8p, i64p]
        L.orc_init.restype = None
        L.orc_tables.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp, dp]
        L.orc_tables.restype = None
        L.orc_accept.argtypes = [ctypes.c_uint32, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_accept.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, i8p, i64p,
                              dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int, i64p, i64p, u64p, u64p,
                              ctypes.c_int]
        L.orc_run.restype = ctypes.c_int
        L.orc_update_weights.argtypes = [ctypes.c_int, i64p, dp]
        L.orc_update_weights.restype = ctypes.c_double
        L.orc_update_weights_ex.argtypes = [ctypes.c_int, i64p, dp, ctypes.c_uint, dp, ctypes.POINTER(ctypes.c_uint8)]
        L.orc_update_weights_ex.restype = ctypes.c_double
        L.orc_update_weights_window.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, i64p, dp,
                                                ctypes.c_uint, dp, ctypes.POINTER(ctypes.c_uint8)]
        L.orc_update_weights_window.restype = ctypes.c_double
        L.orc_tables_window.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_tables_window.restype = None
        L.orc_window_walls.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp]
        L.orc_window_walls.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# --------------------------------------------------------------------------
# Random numbers and lattice
# --------------------------------------------------------------------------
def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    """Philox4x32-10 block (Salmon et al., SC'11) at counter ctr[4], key key[2]."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return [int(v) for v in out]


def num_colours(L: int) -> int:
    return lib().orc_num_colours(L)


def order(L: int) -> np.ndarray:
    """Colour-major visiting order: order[p] = site index x + L(y + Lz)."""
    o = np.zeros(L ** 3, dtype=np.int32)
    lib().orc_order(L, _ptr(o, ctypes.c_int32))
    return o


def energies(L: int, spins: np.ndarray) -> tuple:
    """(E_J, E_Delta, M) of one site-indexed int8 lattice, by full recomputation."""
    s = np.ascontiguousarray(spins, dtype=np.int8)
    out = np.zeros(3, dtype=np.int64)
    lib().orc_energies(L, _ptr(s, ctypes.c_int8), _ptr(out, ctypes.c_int64))
    return int(out[0]), int(out[1]), int(out[2])


def tables(V: int, beta: float, lnW: np.ndarray):
    """Threshold tables (Bp[25], Rp[V+1], Rm[V+1]) of the acceptance rule."""
    lw = np.ascontiguousarray(lnW, dtype=np.float64)
    Bp = np.zeros(25, dtype=np.float64)
    Rp = np.zeros(V + 1, dtype=np.float64)
    Rm = np.zeros(V + 1, dtype=np.float64)
    lib().orc_tables(V, float(beta), _ptr(lw, ctypes.c_double), _ptr(Bp, ctypes.c_double),
                     _ptr(Rp, ctypes.c_double), _ptr(Rm, ctypes.c_double))
    return Bp, Rp, Rm


def tables_window(V: int, beta: float, lnW: np.ndarray, lo: int, hi: int):
    """Threshold tables with the moves out of the window [lo, hi] rejected."""
    lw = np.ascontiguousarray(lnW, dtype=np.float64)
    Bp = np.zeros(25, dtype=np.float64)
    Rp = np.zeros(V + 1, dtype=np.float64)
    Rm = np.zeros(V + 1, dtype=np.float64)
    lib().orc_tables_window(V, float(beta), _ptr(lw, ctypes.c_double), int(lo), int(hi), _ptr(Bp, ctypes.c_double),
                            _ptr(Rp, ctypes.c_double), _ptr(Rm, ctypes.c_double))
    return Bp, Rp, Rm


def accept(u31: int, dEJ: int, d: int, E: int, Bp, Rp, Rm) -> bool:
    return bool(lib().orc_accept(u31, dEJ, d, E, _ptr(Bp, ctypes.c_double), _ptr(Rp, ctypes.c_double),
                                 _ptr(Rm, ctypes.c_double)))


def beta_of(T: float) -> float:
    """beta = 1/T (J = k_B = 1); T = inf gives beta = 0."""
    return 0.0 if math.isinf(T) else 1.0 / T


# --------------------------------------------------------------------------
# A multicanonical job: walkers, histograms, weights
# --------------------------------------------------------------------------
class OracleJob:
    """Walkers [first_walker, first_walker + n_walkers) of one (L, T)
    multicanonical job, held on the host."""

    def __init__(self, L: int, T: float, n_walkers: int, seed: int, lnW=None, n_threads: int = 0,
                 first_walker: int = 0):
        self.L, self.V = L, L ** 3
        self.T, self.beta = T, beta_of(T)
        self.n_walkers, self.seed = n_walkers, seed
        self.n_threads = n_threads
        self.first_walker = first_walker
        self.spins = np.zeros((n_walkers, self.V), dtype=np.int8)
        self.state = np.zeros((n_walkers, 4), dtype=np.int64)
        lib().orc_init(L, seed, first_walker, n_walkers, _ptr(self.spins, ctypes.c_int8), _ptr(self.state, ctypes.c_int64))
        self.lnW = np.zeros(self.V + 1) if lnW is None else np.array(lnW, dtype=np.float64)
        self.lo, self.hi = 0, self.V
        self.hist = np.zeros(self.V + 1, dtype=np.int64)
        self.reset_accum()
        self.threads_used = 0
        self.set_recursion(0)

    def set_recursion(self, flags: int):
        """Weight recursion from now on: 0 plain, bit 0 accumulated pair
        statistics, bit 1 edge extrapolation (orc_update_weights_ex).  Clears
        the accumulated statistics and the visited range."""
        self.recursion = int(flags)
        self.kacc = np.zeros(max(self.V, 1), dtype=np.float64)
        self.seen = np.zeros(self.V + 1, dtype=np.uint8)

    def set_window(self, lo: int, hi: int):
        """Confine the walkers to E_Delta in [lo, hi] (0 <= lo < hi <= V): moves
        out of the window are rejected, the weights outside it become walls
        towards it (orc_window_walls), the recursion and its flatness act on
        the window only, and only measurements inside it are recorded.
        Clears the recursion statistics and the production sums."""
        if not (0 <= lo < hi <= self.V):
            raise ValueError("window must satisfy 0 <= lo < hi <= V")
        self.lo, self.hi = int(lo), int(hi)
        lib().orc_window_walls(self.V, self.beta, self.lo, self.hi, _ptr(self.lnW, ctypes.c_double))
        self.set_recursion(self.recursion)
        self.reset_accum()

    def reset_accum(self):
        self.acc = np.zeros((5, self.V + 1), dtype=np.int64)
        self.sm4_lo = np.zeros(self.V + 1, dtype=np.uint64)
        self.sm4_hi = np.zeros(self.V + 1, dtype=np.uint64)

    def sweep(self, n_sweeps: int, record: bool = False):
        """n_sweeps sweeps of every walker; histogram entries are added to self.hist."""
        self.threads_used = lib().orc_run(
            self.L, self.beta, self.seed, self.first_walker, self.n_walkers, _ptr(self.spins, ctypes.c_int8),
            _ptr(self.state, ctypes.c_int64), _ptr(self.lnW, ctypes.c_double), self.lo, self.hi, int(n_sweeps),
            1 if record else 0, _ptr(self.hist, ctypes.c_int64), _ptr(self.acc, ctypes.c_int64),
            _ptr(self.sm4_lo, ctypes.c_uint64), _ptr(self.sm4_hi, ctypes.c_uint64), self.n_threads)

    def take_hist(self) -> np.ndarray:
        h = self.hist.copy()
        self.hist[:] = 0
        return h

    def update_weights(self, hist: np.ndarray) -> float:
        """MUCA recursion on self.lnW (plain unless set_recursion chose a
        variant); returns the flatness of hist."""
        h = np.ascontiguousarray(hist, dtype=np.int64)
        if self.recursion == 0 and (self.lo, self.hi) == (0, self.V):
            self.seen |= (h > 0).astype(np.uint8)
            return float(lib().orc_update_weights(self.V, _ptr(h, ctypes.c_int64), _ptr(self.lnW, ctypes.c_double)))
        return float(lib().orc_update_weights_window(self.V, self.beta, self.lo, self.hi, _ptr(h, ctypes.c_int64),
                                                     _ptr(self.lnW, ctypes.c_double), self.recursion,
                                                     _ptr(self.kacc, ctypes.c_double), _ptr(self.seen, ctypes.c_uint8)))

    def bin_sums(self) -> Dict[str, list]:
        """Per-bin sums of the recorded measurements as exact Python integers."""
        V = self.V
        sm4 = [int(lo) + (int(hi) << 64) for lo, hi in zip(self.sm4_lo, self.sm4_hi)]
        return {"H": [int(v) for v in self.acc[0]], "SJ": [int(v) for v in self.acc[1]],
                "SJJ": [int(v) for v in self.acc[2]], "SA": [int(v) for v in self.acc[3]],
                "SM2": [int(v) for v in self.acc[4]], "SM4": sm4, "V": V}

    def reweight(self, deltas) -> np.ndarray:
        return reweight(self.V, self.beta, self.lnW, self.bin_sums(), deltas)


# --------------------------------------------------------------------------
# Reweighting (Sec. II, time-series reweighting; Eq. (FieldDerivative), (sph))
# --------------------------------------------------------------------------
def reweight(V: int, beta: float, lnW, sums: Dict[str, list], deltas) -> np.ndarray:
    """Canonical expectation values at (beta, Delta) for each Delta in deltas.

    Time-series reweighting weighs every measurement x by
    exp(-beta Delta E_Delta(x)) / W(E_Delta(x)).  That factor depends on x only
    through E_Delta, so sums over measurements group exactly into per-bin sums:
    bin E carries probability p(E) = w(E) H(E) / sum(w H) with
    w(E) = exp(a(E) - max a), a(E) = -beta Delta E - lnW(E), and within a bin
    the measured sums give exact conditional moments.  Central moments are
    taken as between-bin sums of centred bin means plus the exact within-bin
    variance (H SJJ - SJ^2) / H^2 from integers.

    Returns an array of shape (len(deltas), len(OBS_FIELDS)).
    C_field = d<E_J>/dDelta = -beta cov(E_J, E_Delta)                 (Eq. sph)
    dC_dDelta = beta^2 <(E_J - <E_J>)(E_Delta - <E_Delta>)^2>   (Eq. FieldDerivative applied to C)
    cV = beta^2 Var(E_J + Delta E_Delta) / V, binder_U4 = 1 - <M^4>/(3 <M^2>^2),
    edge_weight = p(first visited bin) + p(last visited bin).
    """
    H = sums["H"]
    bins = [E for E in range(V + 1) if H[E] > 0]
    if not bins:
        raise ValueError("no recorded measurements")
    E = np.array(bins, dtype=np.float64)
    h = np.array([float(H[e]) for e in bins])
    mJ = np.array([sums["SJ"][e] / H[e] for e in bins], dtype=np.float64)
    mJJ = np.array([sums["SJJ"][e] / H[e] for e in bins], dtype=np.float64)
    within = np.array([(H[e] * sums["SJJ"][e] - sums["SJ"][e] ** 2) / (H[e] * H[e]) for e in bins],
                      dtype=np.float64)
    mA = np.array([sums["SA"][e] / H[e] for e in bins], dtype=np.float64)
    mM2 = np.array([sums["SM2"][e] / H[e] for e in bins], dtype=np.float64)
    mM4 = np.array([sums["SM4"][e] / H[e] for e in bins], dtype=np.float64)
    lw = np.asarray(lnW, dtype=np.float64)[bins]

    out = np.zeros((len(deltas), len(OBS_FIELDS)))
    for k, delta in enumerate(deltas):
        delta = float(delta)
        a = -(beta * delta) * E - lw
        w = np.exp(a - a.max())
        p = w * h / np.sum(w * h)
        eJ = np.sum(p * mJ)
        eD = np.sum(p * E)
        dJ = mJ - eJ
        dD = E - eD
        var_ej = np.sum(p * (within + dJ * dJ))
        var_ed = np.sum(p * dD * dD)
        cov = np.sum(p * dJ * dD)
        third = np.sum(p * dJ * dD * dD)
        m2 = np.sum(p * mM2)
        m4 = np.sum(p * mM4)
        var_e = var_ej + 2.0 * delta * cov + delta * delta * var_ed
        u4 = 1.0 - m4 / (3.0 * m2 * m2) if m2 > 0 else float("nan")
        edge = p[0] + p[-1] if len(bins) > 1 else p[0]
        out[k] = (delta, eJ, eD, eJ + delta * eD, np.sum(p * mJJ), var_ej, var_ed,
                  -beta * cov, beta * beta * third, beta * beta * var_e / V,
                  np.sum(p * mA), m2, m4, u4, edge)
    return out


# --------------------------------------------------------------------------
# Analysis on top of reweighting (Sec. II-III): the pseudo-critical point
# Delta*_L (maximum of C(Delta), found by bisection on the zero of dC/dDelta),
# jackknife errors over w subsets each leaving out 1/w of the measurements,
# the reweighted distribution of e_Delta, the equal-height field and the barrier.
# --------------------------------------------------------------------------
def _col(name):
    return OBS_FIELDS.index(name)


def peak(V: int, beta: float, lnW, sums, lo: float, hi: float, tol: float = 1e-11):
    """(Delta*, C*) with Delta* in [lo, hi] where dC/dDelta changes sign from
    + to -; bisection until the bracket is narrower than tol."""
    dc = lambda d: reweight(V, beta, lnW, sums, [d])[0, _col("dC_dDelta")]
    flo, fhi = dc(lo), dc(hi)
    if not (flo > 0 and fhi < 0):
        raise ValueError("dC/dDelta does not change sign from + to - on the bracket")
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if dc(mid) > 0:
            lo = mid
        else:
            hi = mid
    d = 0.5 * (lo + hi)
    return d, float(reweight(V, beta, lnW, sums, [d])[0, _col("C_field")])


def block_sums_difference(total: dict, part: dict) -> dict:
    """Per-bin sums of all measurements except those in `part` (exact integers)."""
    return {k: ([a - b for a, b in zip(total[k], part[k])] if k != "V" else total[k]) for k in total}


def add_sums(a: dict, b: dict) -> dict:
    return {k: ([x + y for x, y in zip(a[k], b[k])] if k != "V" else a[k]) for k in a}


def jackknife(values) -> tuple:
    """Jackknife mean and error of leave-one-block-out estimates (Efron)."""
    v = np.asarray(values, dtype=np.float64)
    w = len(v)
    m = v.mean()
    return float(m), float(math.sqrt((w - 1) / w * np.sum((v - m) ** 2)))


def reweighted_log_hist(V: int, beta: float, lnW, H, delta: float) -> np.ndarray:
    """ln P(E_Delta) at (beta, Delta) from the recorded histogram H: the
    measurements of bin E carry weight exp(-beta Delta E) / W(E); -inf where
    nothing was recorded.  Normalised to sum 1."""
    H = np.asarray([float(h) for h in H])
    E = np.arange(V + 1, dtype=np.float64)
    out = np.full(V + 1, -np.inf)
    seen = H > 0
    a = -(beta * delta) * E[seen] - np.asarray(lnW, dtype=np.float64)[seen] + np.log(H[seen])
    amax = a.max()
    out[seen] = a - (amax + math.log(np.sum(np.exp(a - amax))))
    return out


def two_peaks(lnP: np.ndarray, split: int) -> tuple:
    """(E_low, lnP_low, E_high, lnP_high): the maxima of lnP on [0, split) and
    [split, V]."""
    lo = int(np.argmax(lnP[:split]))
    hi = split + int(np.argmax(lnP[split:]))
    return lo, float(lnP[lo]), hi, float(lnP[hi])


def equal_height(V: int, beta: float, lnW, H, lo: float, hi: float, split: int, tol: float = 1e-11):
    """Delta_eqh in [lo, hi] where the two peaks of P(e_Delta) (maxima below and
    above the bin `split`) have equal height, by bisection on their log ratio
    (which decreases as Delta grows: larger Delta favours small E_Delta), and the
    barrier B = ln(P_max / P_min) / (2 beta Delta_eqh), P_min the minimum of P
    between the two peaks."""
    def diff(d):
        _, a, _, b = two_peaks(reweighted_log_hist(V, beta, lnW, H, d), split)
        return b - a
    if not (diff(lo) > 0 and diff(hi) < 0):
        raise ValueError("peak heights do not cross on the bracket")
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if diff(mid) > 0:
            lo = mid
        else:
            hi = mid
    d = 0.5 * (lo + hi)
    lnP = reweighted_log_hist(V, beta, lnW, H, d)
    e1, p1, e2, p2 = two_peaks(lnP, split)
    pmin = float(np.min(lnP[e1:e2 + 1]))
    barrier = (max(p1, p2) - pmin) / (2.0 * beta * d) if beta > 0 and d != 0 else float("nan")
    return d, barrier
