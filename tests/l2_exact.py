"""Brute-force enumeration of the L=2 Blume-Capel lattice (3^8 = 6561 states).

Independent of the oracle: energies are computed here with numpy rolls on a
(z, y, x) array, straight from Eq. (1) with J = 1 and periodic boundaries.  At
L = 2 the +1 and -1 neighbours along an axis coincide, so each geometric pair
appears twice among the 3V forward bonds.
"""
import itertools
import math

import numpy as np

L = 2
V = 8


def all_states() -> np.ndarray:
    """(6561, 8) int8 array; column i is site i = x + 2y + 4z."""
    return np.array(list(itertools.product((-1, 0, 1), repeat=V)), dtype=np.int8)


def energies(states: np.ndarray):
    s = states.reshape(-1, L, L, L).astype(np.int64)  # axes: state, z, y, x
    ej = -(s * (np.roll(s, -1, axis=3) + np.roll(s, -1, axis=2) + np.roll(s, -1, axis=1))).sum(axis=(1, 2, 3))
    ed = (s * s).sum(axis=(1, 2, 3))
    m = s.sum(axis=(1, 2, 3))
    return ej, ed, m


STATES = all_states()
EJ, ED, M = energies(STATES)


def canonical(beta: float, delta: float) -> dict:
    """Exact canonical expectations at (beta, Delta) by direct summation."""
    e = EJ + delta * ED
    a = -beta * e
    w = np.exp(a - a.max())
    p = w / w.sum()
    mj, md = (p * EJ).sum(), (p * ED).sum()
    cov = (p * (EJ - mj) * (ED - md)).sum()
    third = (p * (EJ - mj) * (ED - md) ** 2).sum()
    me = (p * e).sum()
    m2, m4 = (p * M ** 2).sum(), (p * M.astype(float) ** 4).sum()
    return {
        "mean_EJ": mj, "mean_ED": md, "mean_E": me, "mean_EJ2": (p * EJ.astype(float) ** 2).sum(),
        "var_EJ": (p * (EJ - mj) ** 2).sum(), "var_ED": (p * (ED - md) ** 2).sum(),
        "C_field": -beta * cov, "dC_dDelta": beta * beta * third,
        "cV": beta * beta * (p * (e - me) ** 2).sum() / V,
        "mean_absM": (p * np.abs(M)).sum(), "mean_M2": m2, "mean_M4": m4,
        "binder_U4": 1.0 - m4 / (3.0 * m2 * m2),
    }


def muca_bin_sums(beta: float, lnW: np.ndarray, n: float = 1.0) -> dict:
    """Expected per-bin sums of n measurements drawn exactly from the
    multicanonical distribution pi(x) ~ exp(-beta E_J(x)) W(E_Delta(x))."""
    a = -beta * EJ + lnW[ED]
    w = np.exp(a - a.max())
    p = n * w / w.sum()
    out = {k: [0.0] * (V + 1) for k in ("H", "SJ", "SJJ", "SA", "SM2", "SM4")}
    for E in range(V + 1):
        sel = ED == E
        out["H"][E] = float(p[sel].sum())
        out["SJ"][E] = float((p[sel] * EJ[sel]).sum())
        out["SJJ"][E] = float((p[sel] * EJ[sel].astype(float) ** 2).sum())
        out["SA"][E] = float((p[sel] * np.abs(M[sel])).sum())
        out["SM2"][E] = float((p[sel] * M[sel].astype(float) ** 2).sum())
        out["SM4"][E] = float((p[sel] * M[sel].astype(float) ** 4).sum())
    out["V"] = V
    return out


def ln_g_beta(beta: float) -> np.ndarray:
    """ln sum_{E_J} g(E_J, E_Delta) exp(-beta E_J) for E_Delta = 0..V."""
    out = np.zeros(V + 1)
    for E in range(V + 1):
        sel = ED == E
        a = -beta * EJ[sel]
        out[E] = a.max() + math.log(np.exp(a - a.max()).sum())
    return out
