"""Pins of the oracle against what the paper and mathematics fix, independent of
the oracle's own code: published Philox answers, brute-force enumeration of the
L = 2 lattice, closed forms (E_Delta marginal, beta = 0 density of states,
Ising limit, T -> 0 crossing at Delta_0 = 3), exact detailed balance, and exact
canonical expectation values for the reweighting.
"""
import math
import os

import numpy as np
import pytest

import oracle
from tests import l2_exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------
def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    assert len(rows) == 3
    for r in rows:
        assert oracle.philox4x32_10(r[0:4], r[4:6]) == r[6:10]


def test_initial_spins_uniform_ternary():
    L, n = 8, 16
    job = oracle.OracleJob(L, 2.0, n, seed=123)
    vals, counts = np.unique(job.spins, return_counts=True)
    assert list(vals) == [-1, 0, 1]
    frac = counts / job.spins.size
    assert np.all(np.abs(frac - 1 / 3) < 0.02)
    # different walkers and seeds give different lattices
    assert not np.array_equal(job.spins[0], job.spins[1])
    other = oracle.OracleJob(L, 2.0, 1, seed=124)
    assert not np.array_equal(job.spins[0], other.spins[0])


# --------------------------------------------------------------------------
# Lattice, colouring, energies (Eq. (1))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L", [2, 3, 4, 5, 6, 7, 9])
def test_colour_major_order_is_proper(L):
    V = L ** 3
    order = oracle.order(L)
    assert sorted(order.tolist()) == list(range(V))
    C = oracle.num_colours(L)
    assert C == (2 if L % 2 == 0 else 3)
    # recover colour classes as maximal runs and check no two neighbours share one
    pos = np.empty(V, dtype=np.int64)
    pos[order] = np.arange(V)

    def nbrs(i):
        x, y, z = i % L, (i // L) % L, i // (L * L)
        for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            yield ((x + dx) % L) + L * (((y + dy) % L) + L * ((z + dz) % L))

    # class of a site = its colour under the documented colouring
    def colour(i):
        x, y, z = i % L, (i // L) % L, i // (L * L)
        if L % 2 == 0:
            return (x + y + z) % 2
        f = lambda t: 2 if t == L - 1 else t % 2
        return (f(x) + f(y) + f(z)) % 3

    cols = [colour(int(i)) for i in order]
    assert cols == sorted(cols)  # colour-major
    for i in range(V):
        for j in nbrs(i):
            assert colour(i) != colour(j)
    # within a class, ascending site index (z, then y, then x)
    for c in range(C):
        sites = [int(i) for i in order if colour(int(i)) == c]
        assert sites == sorted(sites)


def test_l2_energies_match_enumeration_and_closed_forms():
    ej = np.array([oracle.energies(2, s)[0] for s in l2_exact.STATES])
    ed = np.array([oracle.energies(2, s)[1] for s in l2_exact.STATES])
    m = np.array([oracle.energies(2, s)[2] for s in l2_exact.STATES])
    assert np.array_equal(ej, l2_exact.EJ)
    assert np.array_equal(ed, l2_exact.ED)
    assert np.array_equal(m, l2_exact.M)
    assert ej.min() == -24 and ej.max() == 24
    # E_Delta marginal: C(8, E) 2^E
    counts = np.bincount(ed, minlength=9)
    assert counts.tolist() == [math.comb(8, E) * 2 ** E for E in range(9)]


@pytest.mark.parametrize("L", [3, 4, 5, 6])
def test_energies_closed_forms(L):
    V = L ** 3
    ones = np.ones(V, dtype=np.int8)
    assert oracle.energies(L, ones) == (-3 * V, V, V)
    assert oracle.energies(L, -ones) == (-3 * V, V, -V)
    assert oracle.energies(L, 0 * ones) == (0, 0, 0)
    if L % 2 == 0:
        x, y, z = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
        idx = (x + L * (y + L * z)).ravel()
        stag = np.empty(V, dtype=np.int8)
        stag[idx] = np.where(((x + y + z) % 2).ravel() == 0, 1, -1)
        assert oracle.energies(L, stag) == (3 * V, V, 0)
    # one flipped spin in the ferromagnet costs 2 * 6 bonds
    s = ones.copy()
    s[0] = -1
    assert oracle.energies(L, s)[0] == -3 * V + 12


# --------------------------------------------------------------------------
# Acceptance: exact detailed balance of the single-site kernel on L = 2
# --------------------------------------------------------------------------
def _acceptance(u_accept, dEJ, d, E, tabs):
    """Exact fraction of u31 in [0, 2^31) accepted (the rule is monotone in u31)."""
    Bp, Rp, Rm = tabs
    lo, hi = 0, 1 << 31  # count = first u that is rejected
    if u_accept(hi - 1, dEJ, d, E, Bp, Rp, Rm):
        return 1.0
    while lo < hi:
        mid = (lo + hi) // 2
        if u_accept(mid, dEJ, d, E, Bp, Rp, Rm):
            lo = mid + 1
        else:
            hi = mid
    return lo / float(1 << 31)


@pytest.mark.parametrize("beta", [0.0, 0.5, 1.11])
def test_detailed_balance_l2(beta):
    rng = np.random.default_rng(7)
    lnW = rng.normal(0.0, 1.5, size=9)
    tabs = oracle.tables(8, beta, lnW)
    states, ej, ed = l2_exact.STATES, l2_exact.EJ, l2_exact.ED
    index = {tuple(s): k for k, s in enumerate(states.tolist())}
    for _ in range(300):
        a = int(rng.integers(len(states)))
        i = int(rng.integers(8))
        sa = states[a].tolist()
        new = [v for v in (-1, 0, 1) if v != sa[i]][int(rng.integers(2))]
        sb = list(sa)
        sb[i] = new
        b = index[tuple(sb)]
        dEJ = int(ej[b] - ej[a])
        d = int(ed[b] - ed[a])
        A_ab = _acceptance(oracle.accept, dEJ, d, int(ed[a]), tabs)
        A_ba = _acceptance(oracle.accept, -dEJ, -d, int(ed[b]), tabs)
        r = math.exp(-beta * dEJ + lnW[ed[b]] - lnW[ed[a]])  # pi(b) / pi(a)
        tol = 2.0 ** -31 + 1e-12
        assert abs(A_ab - min(1.0, r)) <= tol
        assert abs(A_ba - min(1.0, 1.0 / r)) <= tol


# --------------------------------------------------------------------------
# The full colour-major sweep samples exp(-beta E_J) W(E_Delta)
# --------------------------------------------------------------------------
def test_sweep_stationary_distribution_l2():
    beta = 0.5
    rng = np.random.default_rng(11)
    lnW = rng.normal(0.0, 1.0, size=9)
    job = oracle.OracleJob(2, 1.0 / beta, 16, seed=5, lnW=lnW)
    job.sweep(200, record=False)  # equilibrate
    job.sweep(20000, record=True)
    s = job.bin_sums()
    H = np.array(s["H"], dtype=float)
    p_hat = H / H.sum()
    a = -beta * l2_exact.EJ + lnW[l2_exact.ED]
    w = np.exp(a - a.max())
    p = np.array([w[l2_exact.ED == E].sum() for E in range(9)]) / w.sum()
    assert np.all(np.abs(p_hat - p) < 0.004 + 0.05 * p)
    # conditional mean of E_J in each E_Delta bin
    for E in range(9):
        sel = l2_exact.ED == E
        exact = (w[sel] * l2_exact.EJ[sel]).sum() / w[sel].sum()
        if H[E] > 2000:
            assert abs(s["SJ"][E] / H[E] - exact) < 0.25


def test_flat_histogram_at_exact_weights_l2():
    beta = 0.7
    lnW = -l2_exact.ln_g_beta(beta)
    job = oracle.OracleJob(2, 1.0 / beta, 16, seed=9, lnW=lnW)
    job.sweep(200)
    job.take_hist()
    job.sweep(20000)
    h = job.take_hist()
    frac = h / h.sum()
    assert np.all(np.abs(frac - 1.0 / 9) < 0.01)


@pytest.mark.parametrize("L", [3, 5])
def test_flat_histogram_beta0_closed_form(L):
    """At beta = 0 the E_Delta density of states is C(V,E) 2^E for any L, so
    lnW = -ln g gives a flat E_Delta histogram (odd L: 3-colour order)."""
    V = L ** 3
    lnW = np.array([-(math.lgamma(V + 1) - math.lgamma(E + 1) - math.lgamma(V - E + 1) + E * math.log(2))
                    for E in range(V + 1)])
    job = oracle.OracleJob(L, float("inf"), 16, seed=3, lnW=lnW)
    job.sweep(200)
    job.take_hist()
    job.sweep(8000 if L == 3 else 16000)
    h = job.take_hist()
    frac = h / h.sum()
    assert np.all(np.abs(frac - 1.0 / (V + 1)) < 0.25 / (V + 1))


@pytest.mark.parametrize("L,T", [(3, 2.0), (4, 1.0), (5, 1.4182), (6, 0.9)])
def test_tracked_energies_equal_recomputation(L, T):
    rng = np.random.default_rng(L)
    V = L ** 3
    lnW = np.cumsum(rng.normal(0.0, 0.3, size=V + 1))
    job = oracle.OracleJob(L, T, 6, seed=17, lnW=lnW)
    job.sweep(50, record=True)
    for w in range(job.n_walkers):
        assert tuple(job.state[w, :3]) == oracle.energies(L, job.spins[w])
        assert job.state[w, 3] == 50
    assert job.hist.sum() == 6 * 50
    assert job.acc[0].sum() == 6 * 50


def test_thread_split_is_invisible():
    a = oracle.OracleJob(4, 2.0, 7, seed=1, n_threads=1)
    b = oracle.OracleJob(4, 2.0, 7, seed=1, n_threads=3)
    a.sweep(30, record=True)
    b.sweep(30, record=True)
    assert np.array_equal(a.spins, b.spins) and np.array_equal(a.state, b.state)
    assert np.array_equal(a.hist, b.hist) and np.array_equal(a.acc, b.acc)
    assert np.array_equal(a.sm4_lo, b.sm4_lo) and np.array_equal(a.sm4_hi, b.sm4_hi)


# --------------------------------------------------------------------------
# Weight recursion and flatness
# --------------------------------------------------------------------------
def test_recursion_converges_to_beta0_density_of_states():
    L, V = 3, 27
    job = oracle.OracleJob(L, float("inf"), 16, seed=21)
    flat = 0.0
    for it in range(30):
        job.sweep(3000)
        flat = job.update_weights(job.take_hist())
    assert flat > 0.5
    exact = np.array([-math.log(2.0 * (V - E + 1) / E) for E in range(1, V + 1)])
    diffs = np.diff(job.lnW)
    assert np.all(np.abs(diffs - exact) < 0.3), np.max(np.abs(diffs - exact))


def test_recursion_converges_to_exact_weights_l2():
    beta = 0.5
    job = oracle.OracleJob(2, 1.0 / beta, 16, seed=4)
    for it in range(25):
        job.sweep(4000)
        job.update_weights(job.take_hist())
    target = -l2_exact.ln_g_beta(beta)
    assert np.all(np.abs(np.diff(job.lnW) - np.diff(target)) < 0.15)


def test_flatness_special_cases():
    job = oracle.OracleJob(2, 1.0, 1, seed=0)
    lnW = job.lnW.copy()
    assert job.update_weights(np.full(9, 7, dtype=np.int64)) == 1.0
    # a flat histogram shifts every log-weight by the same amount
    assert np.allclose(job.lnW - lnW, -math.log(7.0), atol=0, rtol=0)
    h = np.full(9, 10, dtype=np.int64)
    h[3] = 0
    before = job.lnW.copy()
    assert job.update_weights(h) == 0.0
    assert job.lnW[3] == before[3]
    h = np.array([1, 2, 3, 4, 5, 6, 7, 8, 9], dtype=np.int64)
    assert abs(job.update_weights(h) - 1.0 / 5.0) < 1e-15


# --------------------------------------------------------------------------
# Reweighting against exact canonical values (Sec. II; Eqs. (FieldDerivative), (sph))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("T", [0.8, 2.0])
def test_reweight_exact_l2(T):
    beta = 1.0 / T
    rng = np.random.default_rng(3)
    lnW = rng.normal(0.0, 2.0, size=9)
    sums = l2_exact.muca_bin_sums(beta, lnW, n=1e6)
    deltas = np.linspace(-1.0, 4.5, 23)
    out = oracle.reweight(8, beta, lnW, sums, deltas)
    col = {k: i for i, k in enumerate(oracle.OBS_FIELDS)}
    for r, delta in zip(out, deltas):
        exact = l2_exact.canonical(beta, delta)
        assert r[col["delta"]] == delta
        for k, v in exact.items():
            assert abs(r[col[k]] - v) <= 1e-9 * max(1.0, abs(v)), (k, delta, r[col[k]], v)


def test_field_derivatives_by_finite_differences():
    beta = 1.0 / 1.3
    lnW = np.zeros(9)
    sums = l2_exact.muca_bin_sums(beta, lnW)
    col = {k: i for i, k in enumerate(oracle.OBS_FIELDS)}
    h = 1e-4
    for delta in (1.5, 2.7, 3.3):
        o = oracle.reweight(8, beta, lnW, sums, [delta - h, delta, delta + h])
        dEJ = (o[2, col["mean_EJ"]] - o[0, col["mean_EJ"]]) / (2 * h)
        dC = (o[2, col["C_field"]] - o[0, col["C_field"]]) / (2 * h)
        assert abs(dEJ - o[1, col["C_field"]]) < 1e-6 * max(1, abs(dEJ))
        assert abs(dC - o[1, col["dC_dDelta"]]) < 1e-5 * max(1, abs(dC))


def test_reweight_ising_limit():
    """Delta -> -infinity suppresses vacancies: everything comes from bin E = V."""
    rng = np.random.default_rng(5)
    V = 27
    sums = {"H": [int(v) for v in rng.integers(1, 50, size=V + 1)], "V": V}
    for k in ("SJ", "SJJ", "SA", "SM2", "SM4"):
        sums[k] = [int(v) for v in rng.integers(-100 if k == "SJ" else 0, 1000, size=V + 1)]
    lnW = rng.normal(0.0, 3.0, size=V + 1)
    o = oracle.reweight(V, 0.5, lnW, sums, [-1000.0])[0]
    col = {k: i for i, k in enumerate(oracle.OBS_FIELDS)}
    H = sums["H"][V]
    assert o[col["mean_ED"]] == V
    assert abs(o[col["mean_EJ"]] - sums["SJ"][V] / H) < 1e-12 * abs(sums["SJ"][V] / H)
    assert abs(o[col["mean_M2"]] - sums["SM2"][V] / H) < 1e-12 * abs(sums["SM2"][V] / H)
    assert abs(o[col["C_field"]]) < 1e-150 and abs(o[col["var_ED"]]) < 1e-150
    assert abs(o[col["edge_weight"]] - 1.0) < 1e-12


def test_reweight_canonical_identity():
    """Weights lnW = -beta Delta0 E make the chain canonical at Delta0, so
    reweighting to Delta0 gives plain sample means."""
    L, T, D0 = 3, 1.5, 2.2
    beta = 1.0 / T
    V = L ** 3
    lnW = np.array([-(beta * D0) * E for E in range(V + 1)])
    job = oracle.OracleJob(L, T, 8, seed=31, lnW=lnW)
    job.sweep(50)
    job.sweep(400, record=True)
    s = job.bin_sums()
    o = oracle.reweight(V, beta, lnW, s, [D0])[0]
    col = {k: i for i, k in enumerate(oracle.OBS_FIELDS)}
    n = sum(s["H"])
    assert abs(o[col["mean_EJ"]] - sum(s["SJ"]) / n) < 1e-12 * abs(sum(s["SJ"]) / n)
    assert abs(o[col["mean_ED"]] - sum(E * h for E, h in enumerate(s["H"])) / n) < 1e-12 * V
    assert abs(o[col["mean_M4"]] - sum(s["SM4"]) / n) < 1e-12 * abs(sum(s["SM4"]) / n)


@pytest.mark.parametrize("T", [0.2, 0.25, 0.3])
def test_zero_temperature_crossing_delta0_eq_3(T):
    """At low T the ground state switches from all +-1 (degeneracy 2) to all 0
    at Delta_0 = zJ/2 = 3 (Sec. I); on L = 2 the equal-weight point sits at
    3 + T ln 2 / V up to corrections of order exp(-3 beta)."""
    beta = 1.0 / T
    lnW = -l2_exact.ln_g_beta(beta)  # flat-histogram weights
    sums = l2_exact.muca_bin_sums(beta, lnW)
    col = {k: i for i, k in enumerate(oracle.OBS_FIELDS)}
    lo, hi = 2.5, 3.5
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        eD = oracle.reweight(8, beta, lnW, sums, [mid])[0][col["mean_ED"]]
        if eD > 4.0:
            lo = mid
        else:
            hi = mid
    assert abs(0.5 * (lo + hi) - (3.0 + T * math.log(2.0) / 8)) < T * math.exp(-3.0 * beta)


# --------------------------------------------------------------------------
# Whole pipeline on L = 2: iterate weights, record, reweight vs enumeration
# --------------------------------------------------------------------------
def test_muca_pipeline_l2_matches_enumeration():
    T = 1.0
    beta = 1.0 / T
    job = oracle.OracleJob(2, T, 16, seed=2)
    for it in range(12):
        job.sweep(3000)
        job.update_weights(job.take_hist())
    job.take_hist()
    job.sweep(20000, record=True)
    deltas = [1.0, 2.0, 2.8, 3.0, 3.2, 4.0]
    out = job.reweight(deltas)
    col = {k: i for i, k in enumerate(oracle.OBS_FIELDS)}
    for r, d in zip(out, deltas):
        ex = l2_exact.canonical(beta, d)
        assert abs(r[col["mean_EJ"]] - ex["mean_EJ"]) < 0.2
        assert abs(r[col["mean_ED"]] - ex["mean_ED"]) < 0.1
        assert abs(r[col["C_field"]] - ex["C_field"]) < 0.08 * max(1.0, abs(ex["C_field"]))
        assert abs(r[col["mean_M2"]] - ex["mean_M2"]) < 0.05 * max(1.0, ex["mean_M2"])


# --------------------------------------------------------------------------
# Analysis: peak of C(Delta), jackknife, equal height (Sec. II-III)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("T", [1.0, 1.6])
def test_peak_of_C_matches_dense_exact_scan(T):
    beta = 1.0 / T
    lnW = -l2_exact.ln_g_beta(beta)
    sums = l2_exact.muca_bin_sums(beta, lnW)
    d, c = oracle.peak(8, beta, lnW, sums, 2.0, 4.0)
    grid = np.linspace(2.0, 4.0, 4001)
    cs = np.array([l2_exact.canonical(beta, x)["C_field"] for x in grid])
    k = int(np.argmax(cs))
    assert abs(d - grid[k]) < 1e-3
    assert abs(c - cs[k]) < 1e-6 * abs(cs[k])
    # C is the derivative of <E_J>: at the peak, dC/dDelta vanishes
    assert abs(l2_exact.canonical(beta, d)["dC_dDelta"]) < 1e-6


@pytest.mark.parametrize("T", [0.2, 0.25, 0.3])
def test_equal_height_zero_temperature(T):
    """Two peaks at E_Delta = 0 (all vacancies) and V (no vacancies, degeneracy
    2 at T -> 0): equal height at Delta_0 + T ln 2 / V with Delta_0 = 3 (Sec. I)."""
    beta = 1.0 / T
    lnW = -l2_exact.ln_g_beta(beta)
    sums = l2_exact.muca_bin_sums(beta, lnW, n=1.0)
    d, barrier = oracle.equal_height(8, beta, lnW, sums["H"], 2.5, 3.5, split=4)
    assert abs(d - (3.0 + T * math.log(2.0) / 8)) < T * math.exp(-3.0 * beta)
    assert barrier > 0


def test_reweighted_log_hist_is_exact_canonical_marginal():
    beta, delta = 1.0 / 1.3, 2.7
    lnW = np.random.default_rng(1).normal(0, 1.0, 9)
    sums = l2_exact.muca_bin_sums(beta, lnW)
    lnP = oracle.reweighted_log_hist(8, beta, lnW, sums["H"], delta)
    e = l2_exact.EJ + delta * l2_exact.ED
    w = np.exp(-beta * (e - e.min()))
    exact = np.array([w[l2_exact.ED == E].sum() for E in range(9)]) / w.sum()
    assert np.allclose(np.exp(lnP), exact, rtol=1e-12, atol=0)


def test_jackknife_of_a_linear_statistic_is_the_standard_error():
    x = np.random.default_rng(2).normal(size=20)
    loo = [(x.sum() - xi) / 19 for xi in x]
    m, e = oracle.jackknife(loo)
    assert abs(m - x.mean()) < 1e-12
    assert abs(e - x.std(ddof=1) / math.sqrt(20)) < 1e-12


def _double_well(V, beta, D0, a, s, lnW):
    """A synthetic sample whose reweighted distribution is known in closed form.

    With H(E) = exp(g(E) + beta D0 E + lnW(E)) recorded under weights lnW, the
    reweighted distribution at Delta is ln P(E) = g(E) - beta (Delta - D0) E + const
    (Sec. II: each entry of bin E carries exp(-beta Delta E) / W(E)).  g is the
    symmetric quartic double well -a ((E - c)^2 - s^2)^2 / s^4 about c = V/2,
    with maxima g = 0 at c +- s and g(c) = -a: the two peaks are equal exactly at
    Delta = D0, and ln(P_max / P_min) there is a, P_min taken between the peaks.
    Outside the peaks g falls far below -a."""
    E = np.arange(V + 1, dtype=np.float64)
    c = V / 2
    g = -a * ((E - c) ** 2 - s * s) ** 2 / s ** 4
    return np.exp(g + beta * D0 * E + lnW)


@pytest.mark.parametrize("T,D0,a", [(0.9, 2.964, 7.5), (1.0, 2.944, 3.0), (2.0, 2.523, 11.0)])
def test_equal_height_and_barrier_closed_form(T, D0, a):
    """Sec. III: the barrier is B = ln(P_max / P_min) / (2 beta Delta) at the
    equal-height field.  On the closed-form double well, Delta_eqh = D0 and
    B = a / (2 beta D0); a wrong normalisation, sign of the weights or range of
    P_min fails."""
    beta = 1.0 / T
    V, s = 60, 12
    lnW = np.random.default_rng(7).normal(0.0, 2.0, size=V + 1) - 0.4 * beta * D0 * np.arange(V + 1)
    H = _double_well(V, beta, D0, a, s, lnW)
    d, barrier = oracle.equal_height(V, beta, lnW, list(H), D0 - 0.05, D0 + 0.05, split=V // 2)
    assert abs(d - D0) < 1e-9
    assert abs(barrier - a / (2.0 * beta * D0)) < 1e-9 * (a / (2.0 * beta * D0))
    lnP = oracle.reweighted_log_hist(V, beta, lnW, list(H), D0)
    assert int(np.argmax(lnP[: V // 2])) == V // 2 - s and int(np.argmax(lnP[V // 2:])) == s


def _exact_l2_log_hist(beta, delta):
    """ln P(E_Delta) at (beta, Delta) on L = 2, summed over all 3^8 states."""
    a = -beta * (l2_exact.EJ + delta * l2_exact.ED)
    w = np.exp(a - a.max())
    P = np.array([w[l2_exact.ED == E].sum() for E in range(9)])
    return np.log(P / P.sum())


@pytest.mark.parametrize("T", [0.25, 0.5, 1.0])
def test_barrier_exact_l2(T):
    """The equal-height field and the barrier of Sec. III on L = 2 against the
    enumeration: the field where the maxima of P(E_Delta) below and above
    E_Delta = 4 are equal (found here by bisection on the exact distribution),
    and ln(P_max / P_min) / (2 beta Delta) with P_min between the peaks."""
    beta = 1.0 / T
    lnW = -l2_exact.ln_g_beta(beta)
    sums = l2_exact.muca_bin_sums(beta, lnW, n=1.0)
    d_o, b_o = oracle.equal_height(8, beta, lnW, sums["H"], 2.5, 3.5, split=4)
    lo, hi = 2.5, 3.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        p = _exact_l2_log_hist(beta, mid)
        if p[4:].max() > p[:4].max():
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-13:
            break
    d_x = 0.5 * (lo + hi)
    p = _exact_l2_log_hist(beta, d_x)
    e1, e2 = int(np.argmax(p[:4])), 4 + int(np.argmax(p[4:]))
    b_x = (max(p[e1], p[e2]) - p[e1:e2 + 1].min()) / (2.0 * beta * d_x)
    assert abs(d_o - d_x) < 1e-9
    assert abs(b_o - b_x) < 1e-9 * max(1.0, abs(b_x))


def test_sum_of_m4_carries_past_64_bits():
    """The per-bin sum of M^4 is kept in 128 bits (Sec. II reweighting of <M^4>).
    A frozen ordered lattice (L = 30, all spins +1, T = 0.05: every move costs at
    least exp(-120), so only u31 = 0 would accept) records M = V after every
    sweep: the sum is exactly n V^4, past 2^64 several times over."""
    L, T, nw, sweeps = 30, 0.05, 4, 48
    V = L ** 3
    job = oracle.OracleJob(L, T, nw, seed=77)
    job.spins[:] = 1
    job.state[:] = [-3 * V, V, V, 0]
    job.sweep(sweeps, record=True)
    assert np.all(job.spins == 1) and np.all(job.state[:, :3] == [-3 * V, V, V])
    n = nw * sweeps
    s = job.bin_sums()
    assert s["H"][V] == n and sum(s["H"]) == n
    assert s["SM4"][V] == n * V ** 4 and (n * V ** 4) >> 64 == 5
    assert s["SM2"][V] == n * V * V and s["SA"][V] == n * V and s["SJ"][V] == -3 * V * n
    assert int(job.sm4_hi[V]) == 5 and int(job.sm4_lo[V]) == (n * V ** 4) & (2 ** 64 - 1)


# --------------------------------------------------------------------------
# A job's E_Delta window (the reading that maps a Delta range to [lo, hi])
# --------------------------------------------------------------------------
def test_window_tables_confine_and_walls_pull_in():
    """Moves out of [lo, hi] are rejected whatever the random number; outside
    the window the walls accept every move towards it, whatever dE_J."""
    V, beta, lo, hi = 64, 1.0 / 0.9, 20, 40
    lnW = np.random.default_rng(4).normal(0.0, 1.0, size=V + 1)
    oracle.OracleJob(4, 0.9, 1, 0, lnW=lnW)  # builds the library
    job = oracle.OracleJob(4, 0.9, 1, 0, lnW=lnW)
    job.set_window(lo, hi)
    kappa = 12 * beta + math.log(2 * V) + 1
    assert np.allclose(np.diff(job.lnW[hi:]), -kappa) and np.allclose(np.diff(job.lnW[:lo + 1]), kappa)
    assert np.array_equal(job.lnW[lo:hi + 1], lnW[lo:hi + 1])
    Bp, Rp, Rm = oracle.tables_window(V, beta, job.lnW, lo, hi)
    assert Rp[hi] == 0.0 and Rm[lo] == 0.0
    for dEJ in range(-12, 13):
        assert not oracle.accept(0, dEJ, +1, hi, Bp, Rp, Rm)      # up from the top edge
        assert not oracle.accept(0, dEJ, -1, lo, Bp, Rp, Rm)      # down from the bottom edge
        for E in (hi + 1, hi + 7, V):
            assert oracle.accept(2 ** 31 - 1, dEJ, -1, E, Bp, Rp, Rm)   # down towards the window
        for E in (0, lo - 5, lo - 1):
            assert oracle.accept(2 ** 31 - 1, dEJ, +1, E, Bp, Rp, Rm)   # up towards the window
    # inside the window the tables are the plain ones
    B0, P0, M0 = oracle.tables(V, beta, job.lnW)
    assert np.array_equal(Bp, B0)
    assert np.array_equal(Rp[lo:hi], P0[lo:hi]) and np.array_equal(Rm[lo + 1:hi + 1], M0[lo + 1:hi + 1])


def test_window_stationary_distribution_l2():
    """Confined to E_Delta in [2, 6], the sweep samples exp(-beta E_J) W(E_Delta)
    restricted to the window and renormalised (enumeration), and records
    nothing outside it."""
    beta, lo, hi = 0.5, 2, 6
    lnW = np.random.default_rng(12).normal(0.0, 1.0, size=9)
    job = oracle.OracleJob(2, 1.0 / beta, 16, seed=6, lnW=lnW)
    job.set_window(lo, hi)
    job.sweep(50)
    assert np.all((job.state[:, 1] >= lo) & (job.state[:, 1] <= hi)), "walkers did not enter the window"
    job.take_hist()
    job.sweep(20000, record=True)
    h = job.take_hist()
    assert h[:lo].sum() == 0 and h[hi + 1:].sum() == 0
    s = job.bin_sums()
    assert s["H"] == list(h)
    a = -beta * l2_exact.EJ + lnW[l2_exact.ED]
    w = np.exp(a - a.max())
    p = np.array([w[l2_exact.ED == E].sum() for E in range(9)])
    p[:lo] = 0.0
    p[hi + 1:] = 0.0
    p /= p.sum()
    assert np.all(np.abs(h / h.sum() - p) < 0.004 + 0.05 * p)


@pytest.mark.parametrize("lo,hi", [(30, 70), (90, 125), (0, 20)])
def test_window_flat_histogram_beta0_closed_form(lo, hi):
    """At beta = 0 the E_Delta density of states is C(V,E) 2^E; its inverse as
    weights inside a window gives a flat histogram over that window, and
    walkers that start outside (random lattices sit near E_Delta = 2V/3 = 83)
    enter it through the walls."""
    L = 5
    V = L ** 3
    lnW = -np.array([math.log(math.comb(V, E)) + E * math.log(2.0) for E in range(V + 1)])
    job = oracle.OracleJob(L, float("inf"), 32, seed=21, lnW=lnW)
    job.set_window(lo, hi)
    job.sweep(40)
    assert np.all((job.state[:, 1] >= lo) & (job.state[:, 1] <= hi))
    job.take_hist()
    job.sweep(6000)
    h = job.take_hist()
    assert h[:lo].sum() == 0 and h[hi + 1:].sum() == 0
    frac = h[lo:hi + 1] / h.sum()
    n = hi - lo + 1
    assert np.all(np.abs(frac - 1.0 / n) < 0.25 / n), frac * n


def test_window_recursion_converges_to_restricted_density_of_states():
    """beta = 0, L = 3, window [6, 20]: the plain recursion from flat weights
    converges, inside the window, to -ln(C(V,E) 2^E) up to a constant; the
    walls outside follow the edges."""
    L, lo, hi = 3, 6, 20
    V = L ** 3
    job = oracle.OracleJob(L, float("inf"), 16, seed=8)
    job.set_window(lo, hi)
    for _ in range(40):
        job.sweep(2000)
        job.update_weights(job.take_hist())
    exact = -np.array([math.log(math.comb(V, E)) + E * math.log(2.0) for E in range(V + 1)])
    d = np.diff(job.lnW[lo:hi + 1]) - np.diff(exact[lo:hi + 1])
    assert np.all(np.abs(d) < 0.12), d
    kappa = math.log(2 * V) + 1
    assert np.allclose(np.diff(job.lnW[hi:]), -kappa) and np.allclose(np.diff(job.lnW[:lo + 1]), kappa)


@pytest.mark.parametrize("flags", [0, 3])
def test_full_window_is_no_window(flags):
    """The window [0, V] changes nothing: same chain, same weights bit for bit."""
    L, T = 3, 1.4
    a = oracle.OracleJob(L, T, 6, seed=3)
    b = oracle.OracleJob(L, T, 6, seed=3)
    a.set_recursion(flags)
    b.set_recursion(flags)
    b.set_window(0, L ** 3)
    for _ in range(4):
        a.sweep(30)
        b.sweep(30)
        ha, hb = a.take_hist(), b.take_hist()
        assert np.array_equal(ha, hb)
        assert a.update_weights(ha) == b.update_weights(hb)
        assert a.lnW.tobytes() == b.lnW.tobytes()
    assert np.array_equal(a.spins, b.spins)
