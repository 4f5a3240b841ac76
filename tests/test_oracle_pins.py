"""Pins of the FP64 oracle to facts fixed outside it (CPU only).

Each test checks the oracle against something the paper or the mathematics
fixes: the printed worked example, the queueing quadratic, the SCALE bound,
closed-form optima (Lambert-W, EE water-filling), the Dinkelbach and SCA
propositions, finite-difference stationarity (KKT), exact scaling invariance,
permutation equivariance and brute force on tiny instances.
"""
import math
import os

import numpy as np
import pytest
from scipy.special import lambertw

import oracle
import synth
from tests import refeval
from tests.drops_util import custom_drop, psi_of

GOLD = os.path.join(os.path.dirname(__file__), "golden")

CONVERGE = dict(fixed_count=0, sweeps_per_dinkelbach=200000, tol_dual=1e-14,
                tol_dinkelbach=1e-13, max_dinkelbach=60)


def read_kv(name):
    out = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


# ---------------------------------------------------------------- Psi (C9)

def test_min_rate_worked_example():
    """Sec. VIII: 125 packets/s, 25 packets queued, 1024-bit packets -> 4.18."""
    g = read_kv("min_rate_worked_example.txt")
    lam, q = g["lambda_pkt_s"], g["queue_len_pkt"]
    T = q / lam  # T_k = q_k / lambda_k (Sec. II-A)
    assert T == pytest.approx(0.2, rel=1e-15)
    psi = oracle.min_rate(lam * g["packet_bits"], T, g["packet_bits"], g["bw_hz"])
    digits = int(g["printed_digits"])
    assert float(f"{psi:.{digits}g}") == g["printed_min_rate"]


def test_min_rate_is_smaller_root_of_delay_quadratic():
    """Psi = zbar/(X B_n) with X the smaller root of
    lambda X^2 - X(2+2 lambda T) + 2T = 0 (Sec. II-B)."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        rate = rng.uniform(8e3, 2e6)
        T = rng.uniform(1e-3, 2.0)
        zbar = rng.choice([256.0, 1024.0, 12000.0])
        bw = rng.choice([15e3, 31.25e3, 180e3])
        psi = oracle.min_rate(rate, T, zbar, bw)
        lam = rate / zbar
        X = zbar / (psi * bw)
        resid = lam * X * X - X * (2 + 2 * lam * T) + 2 * T
        assert abs(resid) <= 1e-10 * 2 * T
        other = (2 + 2 * lam * T) / lam - X  # sum of roots
        assert X <= other * (1 + 1e-12)
        assert psi == pytest.approx(refeval.min_rate_quadratic(rate, T, zbar, bw), rel=1e-9)


def test_min_rate_limits():
    """Long delay budgets need the arrival bit rate; short ones one packet per T."""
    zbar, bw = 1024.0, 180e3
    lam = 1000.0
    T_long = 1e6 / lam
    psi = oracle.min_rate(lam * zbar, T_long, zbar, bw)
    assert psi * bw == pytest.approx(lam * zbar, rel=1e-6)
    T_short = 1e-7 / lam
    psi = oracle.min_rate(lam * zbar, T_short, zbar, bw)
    assert psi * bw == pytest.approx(zbar / T_short, rel=1e-5)


# ---------------------------------------------------------- SCALE bound

@pytest.mark.parametrize("z0", [1e-3, 0.1, 1.0, 7.5, 1e3, 1e6])
def test_scale_bound_tight_lower_and_tangent(z0):
    a, b = oracle.scale_coeffs(z0)
    assert a * math.log2(z0) + b == pytest.approx(math.log2(1 + z0), rel=1e-14, abs=1e-15)
    zs = np.logspace(-6, 8, 400)
    lower = a * np.log2(zs) + b
    assert (lower <= np.log2(1 + zs) + 1e-12).all()
    # equal derivatives at z0: alpha/(z ln2) = 1/((1+z) ln2)
    assert a / z0 == pytest.approx(1.0 / (1.0 + z0), rel=1e-14)


# ------------------------------------------------------------ SIC margin

def test_sic_margin_sign_is_normalised_gain_order():
    """Omega <= 0 exactly when the raw-stronger user also has the larger
    Gamma/(sigma+ICI) (Sec. II-A, eq. SIC_linear)."""
    rng = np.random.default_rng(2)
    sg = 7e-16
    agree = 0
    for _ in range(5000):
        gs, gw = np.sort(10.0 ** rng.uniform(-14, -6, 2))[::-1]
        ici_s, ici_w = 10.0 ** rng.uniform(-18, -9, 2)
        om = oracle.sic_margin(gs, gw, ici_s, ici_w, sg)
        gts, gtw = gs / (sg + ici_s), gw / (sg + ici_w)
        assert (om <= 0) == (gts >= gtw)
        assert -1.0 <= om <= 1.0
        agree += om <= 0
    assert 0 < agree < 5000
    # no inter-cell interference: always decodable in raw order
    for _ in range(100):
        gs, gw = np.sort(10.0 ** rng.uniform(-14, -6, 2))[::-1]
        assert oracle.sic_margin(gs, gw, 0.0, 0.0, sg) <= 0.0


# ------------------------------------------------ closed-form special cases

def _lambert_opt(a, P0, eta, pmask):
    """argmax_p log2(1+a p)/(P0 + eta p) on [0, pmask]."""
    y = math.exp(lambertw((a * P0 / eta - 1.0) / math.e).real + 1.0)
    p = min(max((y - 1.0) / a, 0.0), pmask)
    return p, math.log2(1 + a * p) / (P0 + eta * p)


@pytest.mark.parametrize("pmax", [39.8, 0.05])
def test_single_link_matches_lambert_w(pmax):
    """M=N=K=1 elastic: the EE optimum has the Lambert-W closed form."""
    sg, g = 1e-15, 1e-12
    d = custom_drop(np.full((1, 1, 1), g), pmax=[pmax], eta=[4.0], noise=sg, l=1)
    r = oracle.solve(d, oracle.Params(**CONVERGE))
    P0 = refeval.static_power(d)
    p_star, e_star = _lambert_opt(float(np.float32(g)) / sg, P0, 4.0, pmax)
    assert r.ee == pytest.approx(e_star, rel=1e-10)
    assert r.slot_power[0, 0, 0] == pytest.approx(p_star, rel=1e-8)
    assert r.sel[0, 0, 0] == 0 and r.rrh_of_user[0] == 0
    assert r.status_flags & oracle.NOT_CONVERGED == 0


def _water_filling(d):
    """EE-optimal OFDMA powers for M=1, l=1, all elastic (textbook):
    each subcarrier to its best user, p_n = [1/(E eta ln2) - sigma/Gamma_n]_0^pmask,
    E the root of F(E) = sum log2(1+Gamma p/sigma) - E (P0 + eta sum p)."""
    G = d.gain[0].astype(np.float64)
    best = G.argmax(axis=1)
    gn = G[np.arange(d.N), best]
    P0, eta, pmask, sg = refeval.static_power(d), d.eta[0], d.pmax_w[0] / d.N, d.noise_w

    def powers(E):
        return np.clip(1.0 / (E * eta * math.log(2)) - sg / gn, 0.0, pmask)

    def F(E):
        p = powers(E)
        return np.log2(1 + gn * p / sg).sum() - E * (P0 + eta * p.sum())

    lo, hi = 1e-6, 1e6
    for _ in range(300):
        mid = math.sqrt(lo * hi)
        if F(mid) > 0:
            lo = mid
        else:
            hi = mid
    E = 0.5 * (lo + hi)
    return best, powers(E), E


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ofdma_single_rrh_matches_water_filling(seed):
    rng = np.random.default_rng(100 + seed)
    N, K = 8, 4
    gain = 10.0 ** rng.uniform(-13.5, -12.0, (1, N, K))
    d = custom_drop(gain, pmax=[2.0], eta=[4.0], noise=1e-15, l=1)
    best, p_wf, E_wf = _water_filling(d)
    r = oracle.solve(d, oracle.Params(**CONVERGE))
    assert r.ee == pytest.approx(E_wf, rel=1e-9)
    for n in range(N):
        if p_wf[n] > 0:
            assert r.sel[0, n, 0] == best[n]
            assert r.slot_power[0, n, 0] == pytest.approx(p_wf[n], rel=1e-7)
        else:
            assert r.sel[0, n, 0] == -1 or r.slot_power[0, n, 0] <= 1e-12
    # Prop. 1: E^i strictly increases while F_i > 0, and F_i decreases (Lemma 1)
    E, F = r.trace_E, r.trace_F
    for i in range(len(E) - 1):
        if F[i] > 1e-12 * r.rate_sum:
            assert E[i + 1] > E[i]
            assert F[i + 1] < F[i]


def test_dinkelbach_parametric_function():
    """Theorem 1 / Lemma 1: F(E) = max_p R - E P is strictly decreasing and
    vanishes at the optimal energy efficiency."""
    rng = np.random.default_rng(7)
    gain = 10.0 ** rng.uniform(-13.5, -12.0, (1, 6, 3))
    d = custom_drop(gain, pmax=[2.0], eta=[4.0], noise=1e-15, l=1)
    r = oracle.solve(d, oracle.Params(**CONVERGE))
    Estar = r.ee
    st = oracle.State(d, oracle.Params(**CONVERGE))
    Fs = []
    grid = Estar * np.array([0.5, 0.8, 0.95, 1.0, 1.05, 1.3, 2.0])
    for E in grid:
        st.set_E(E)
        for v in range(200000):
            if st.sweep(v, True) < 1e-14:
                break
        R, P, _, _ = st.evaluate()
        Fs.append(R - E * P)
    Fs = np.array(Fs)
    assert (np.diff(Fs) < 0).all()
    assert abs(Fs[3]) <= 1e-9 * Estar * 10
    assert (Fs[:3] > 0).all() and (Fs[4:] < 0).all()


def test_sca_rounds_never_decrease_objective():
    """Prop. 2: with alpha/beta refitted only after the inner loop converges,
    the true objective R - E P is non-decreasing over SCALE rounds, and the
    SCALE surrogate never exceeds the true rate."""
    rng = np.random.default_rng(3)
    N, K = 4, 2
    gain = 10.0 ** rng.uniform(-13, -11, (1, N, K))
    d = custom_drop(gain, pmax=[1000.0], eta=[4.0], noise=1e-15, l=2)
    st = oracle.State(d, oracle.Params(**CONVERGE))
    st.set_E(50.0)
    st.reset_scale()
    objs = []
    v = 0
    for s in range(25):
        st.sweep(v, True)  # refit at the current point, then the inner loop
        v += 1
        for _ in range(200000):
            d_ = st.sweep(v, False)
            v += 1
            if d_ < 1e-14:
                break
        R, P, Rh, _ = st.evaluate()
        assert Rh <= R + 1e-9 * abs(R)
        objs.append(R - 50.0 * P)
    objs = np.array(objs)
    assert (np.diff(objs) >= -1e-10 * np.abs(objs[1:])).all()
    assert objs[-1] > objs[0]


def _two_cell_drop(seed):
    """Two RRHs, each with two nearby users; cross gains 15 dB weaker, so both
    cells are active on every subcarrier and interfere with each other.  A
    user's cross gain is its own gain times one factor per subcarrier, so on
    every subcarrier the normalised-gain order of a cell's users is their
    raw-gain order: C14 holds for every pair and both users of a cell can
    share a subcarrier."""
    rng = np.random.default_rng(seed)
    M, N, K = 2, 3, 4
    own = np.array([0, 0, 1, 1])
    gain = np.empty((M, N, K))
    cross = 10.0 ** (-1.5 + rng.uniform(-0.2, 0.2, N))
    for k in range(K):
        g = 10.0 ** (-11.5 + rng.uniform(-0.5, 0.5, N))
        gain[own[k], :, k] = g
        gain[1 - own[k], :, k] = g * cross
    return custom_drop(gain, pmax=[6.0, 6.0], eta=[4.0, 2.0], noise=1e-15, l=2)


@pytest.mark.parametrize("seed", [11, 12])
def test_stationarity_by_finite_differences(seed):
    """KKT: at a converged sweep fixed point (fixed E, slack budget, no active
    SIC multiplier) every interior power is a stationary point of R - E P, with
    intra-cell NOMA and inter-cell interference both present.  At the same
    point the selection metric of a selected user equals its Lagrangian
    surplus w mu [log2(1+gamma) - gamma/((1+gamma) ln 2)], which follows from
    stationarity of the per-triple maximisation."""
    d = _two_cell_drop(seed)
    st = oracle.State(d, oracle.Params(**CONVERGE))
    E = 20.0
    st.set_E(E)
    for v in range(200000):
        if st.sweep(v, True) < 1e-15:
            break
    sel, p, xi, zeta, zs = st.slots()
    assert (xi == 0).all() and (zs == 0).all()
    assert (sel[0] >= 0).any() and (sel[1] >= 0).any()  # both cells active
    H = st.lagrangian_metric()
    P = refeval.dense_from_slots(d, sel, p)
    G = d.gain.astype(np.float64)
    tot = P.sum(axis=2)
    N = d.N
    pmask = d.pmax_w / N
    checked = 0
    for idx in zip(*np.nonzero(sel >= 0)):
        m, n, s = idx
        if not (1e-9 * pmask[m] < p[idx] < pmask[m] * (1 - 1e-6)):
            continue
        h = 1e-6 * p[idx]
        vals = []
        for sgn in (+1, -1):
            q = p.copy()
            q[idx] += sgn * h
            st.set_powers(q)
            R, Pw, _, _ = st.evaluate()
            vals.append(R - E * Pw)
        st.set_powers(p)
        grad = (vals[0] - vals[1]) / (2 * h)
        scale = 1.0 / (math.log(2) * p[idx])  # size of one term of the gradient
        assert abs(grad) <= 1e-5 * scale, (idx, grad, scale)
        # SINR of this user from the independent evaluator's definition
        k = sel[idx]
        users = [u for u in sel[m, n] if u >= 0]
        ici = {u: sum(tot[j, n] * G[j, n, u] for j in range(d.M) if j != m) for u in users}
        gt = {u: G[m, n, u] / (d.noise_w + ici[u]) for u in users}
        before = sum(P[m, n, u] for u in users if gt[u] > gt[k] or (gt[u] == gt[k] and u < k))
        gam = P[m, n, k] * G[m, n, k] / (d.noise_w + ici[k] + G[m, n, k] * before)
        surplus = math.log2(1 + gam) - gam / ((1 + gam) * math.log(2))
        assert H[m, n, k] == pytest.approx(surplus, rel=1e-6)
        checked += 1
    assert checked >= 6


def _near_far_weighted_drop(seed):
    """Two cells with a near and a far user each; the far users carry the larger
    priority weight, which makes NOMA pairs worthwhile."""
    rng = np.random.default_rng(seed)
    M, N, K = 2, 2, 4
    own, near = [0, 0, 1, 1], [1, 0, 1, 0]
    gain = np.empty((M, N, K))
    for m in range(M):
        for k in range(K):
            base = (-10.5 if near[k] else -12.5) if own[k] == m else -13.5
            gain[m, :, k] = 10.0 ** (base + rng.uniform(-0.3, 0.3, N))
    w = np.array([[0.2 if near[k] else 1.0 for k in range(K)] for m in range(M)])
    return custom_drop(gain, pmax=[6.0, 6.0], eta=[4.0, 2.0], noise=1e-15, l=2), w


def test_sic_multiplier_stationarity():
    """With fixed positive C14 multipliers (step 0), the sweep fixed point is a
    stationary point of R - E P - sum zeta~ Omega/nu (nu at the point): the SIC
    prices enter with the right sign, split into numerator and denominator."""
    d, w = _near_far_weighted_drop(2)
    prm = oracle.Params(**dict(CONVERGE, step0=0.0))
    st = oracle.State(d, prm, weight=w)
    E = 20.0
    st.set_E(E)
    for v in range(20000):
        if st.sweep(v, True) < 1e-15:
            break
    sel, p, xi, zeta, zs = st.slots()
    # positive multipliers on every co-scheduled pair
    zs = np.zeros_like(zs)
    M, N, L = sel.shape
    npairs = 0
    for m in range(M):
        for n in range(N):
            for a in range(L):
                for b in range(L):
                    if a != b and sel[m, n, a] >= 0 and sel[m, n, b] >= 0:
                        zs[m, n, a, b] = 0.3
                        npairs += 1
    assert npairs >= 4
    st.set_multipliers(zs=zs)
    for v in range(200000):
        if st.sweep(v, True) < 1e-15:
            break
    sel2, p, xi, zeta, zs2 = st.slots()
    assert np.array_equal(sel2, sel) and np.array_equal(zs2, zs)
    G = d.gain.astype(np.float64)
    sg = d.noise_w

    def sic_term(pw):
        P = refeval.dense_from_slots(d, sel, pw)
        tot = P.sum(axis=2)
        acc = 0.0
        for m in range(M):
            for n in range(N):
                for a in range(L):
                    for b in range(a + 1, L):
                        ka, kb = sel[m, n, a], sel[m, n, b]
                        if ka < 0 or kb < 0:
                            continue
                        s_, w_ = (ka, kb) if (G[m, n, ka], -ka) >= (G[m, n, kb], -kb) else (kb, ka)
                        ici = lambda k: sum(tot[j, n] * G[j, n, k] for j in range(M) if j != m)
                        om = (G[m, n, w_] * (sg + ici(s_)) - G[m, n, s_] * (sg + ici(w_)))
                        acc += zs[m, n, a, b] * om / nu[(m, n, a, b)]
        return acc

    P0 = refeval.dense_from_slots(d, sel, p)
    tot0 = P0.sum(axis=2)
    nu = {}
    for m in range(M):
        for n in range(N):
            for a in range(L):
                for b in range(a + 1, L):
                    ka, kb = sel[m, n, a], sel[m, n, b]
                    if ka < 0 or kb < 0:
                        continue
                    s_, w_ = (ka, kb) if (G[m, n, ka], -ka) >= (G[m, n, kb], -kb) else (kb, ka)
                    ici = lambda k: sum(tot0[j, n] * G[j, n, k] for j in range(M) if j != m)
                    nu[(m, n, a, b)] = G[m, n, w_] * (sg + ici(s_)) + G[m, n, s_] * (sg + ici(w_))
    pmask = d.pmax_w / N
    checked = 0
    for idx in zip(*np.nonzero(sel >= 0)):
        if not (1e-9 * pmask[idx[0]] < p[idx] < pmask[idx[0]] * (1 - 1e-6)):
            continue
        h = 1e-6 * p[idx]
        vals = []
        for sgn in (+1, -1):
            q = p.copy()
            q[idx] += sgn * h
            st.set_powers(q)
            R, Pw, _, _ = st.evaluate()
            vals.append(R - E * Pw - sic_term(q))
        st.set_powers(p)
        grad = (vals[0] - vals[1]) / (2 * h)
        assert abs(grad) <= 1e-5 / (math.log(2) * p[idx]), (idx, grad)
        checked += 1
    assert checked >= 4


# -------------------------------------------------------------- metamorphic

def _solve2(d, gain=None, **kw):
    return oracle.solve(d, oracle.Params(sweeps_per_dinkelbach=60, **kw), gain=gain)


def test_gain_and_noise_scaling_invariance_exact():
    d = synth.make_drop(synth.CFG2, 5, 0)
    r0 = _solve2(d)
    d2 = synth.make_drop(synth.CFG2, 5, 0)
    d2.gain = d.gain * np.float32(2.0 ** 10)
    d2.noise_w = d.noise_w * 2.0 ** 10
    r1 = _solve2(d2)
    assert r0.ee == r1.ee
    assert np.array_equal(r0.sel, r1.sel)
    assert np.array_equal(r0.slot_power, r1.slot_power)
    assert np.array_equal(r0.rrh_of_user, r1.rrh_of_user)


def test_user_permutation_equivariance():
    d = synth.make_drop(synth.CFG2, 6, 0)
    perm = np.random.default_rng(0).permutation(d.K)
    inv = np.argsort(perm)
    r0 = _solve2(d)
    dp = synth.make_drop(synth.CFG2, 6, 0)
    dp.gain = np.ascontiguousarray(d.gain[:, :, perm])
    dp.user_type = d.user_type[perm]
    dp.arrival_bps = d.arrival_bps[perm]
    dp.delay_s = d.delay_s[perm]
    r1 = _solve2(dp)
    assert r0.near_ties == 0
    assert r1.ee == pytest.approx(r0.ee, rel=1e-10)
    assert np.array_equal(r1.rrh_of_user, r0.rrh_of_user[perm])
    mapped = np.where(r1.sel >= 0, perm[np.maximum(r1.sel, 0)], -1)
    assert np.array_equal(mapped, r0.sel)
    np.testing.assert_allclose(r1.slot_power, r0.slot_power, rtol=1e-8, atol=1e-15)
    np.testing.assert_allclose(r1.user_rate, r0.user_rate[perm], rtol=1e-8, atol=1e-12)
    assert inv is not None


def test_subcarrier_and_lpn_permutation_equivariance():
    d = synth.make_drop(synth.CFG2, 7, 0)
    r0 = _solve2(d)
    pn = np.random.default_rng(1).permutation(d.N)
    dn = synth.make_drop(synth.CFG2, 7, 0)
    dn.gain = np.ascontiguousarray(d.gain[:, pn, :])
    r1 = _solve2(dn)
    assert r1.ee == pytest.approx(r0.ee, rel=1e-10)
    assert np.array_equal(r1.sel, r0.sel[:, pn, :])
    pm = np.array([0, 3, 1, 4, 2])  # keep the HPN at index 0
    dm = synth.make_drop(synth.CFG2, 7, 0)
    dm.gain = np.ascontiguousarray(d.gain[pm])
    dm.pmax_w = d.pmax_w[pm]
    dm.eta = d.eta[pm]
    r2 = _solve2(dm)
    assert r2.ee == pytest.approx(r0.ee, rel=1e-10)
    assert np.array_equal(r2.sel, r0.sel[pm])
    a0 = r0.rrh_of_user
    mapped = np.where(r2.rrh_of_user >= 0, pm[np.maximum(r2.rrh_of_user, 0)], -1)
    assert np.array_equal(mapped, a0)


# ------------------------------------------------------------ feasibility

@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_output_feasible_and_consistent(seed):
    """Outputs meet C1, C4, C5, C8 and the budget, and the reported EE and rates
    agree with an independent evaluation of the returned allocation."""
    d = synth.make_drop(synth.CFG2, seed, 0)
    r = oracle.solve(d, oracle.Params())
    P = refeval.dense_from_slots(d, r.sel, r.slot_power)
    # the drop has eight streaming users: C12, C13 and C14 hold too
    ok = refeval.feasibility(d, P, d.l, psi=psi_of(d), qos_rel=1e-6, tol=1e-6)
    assert all(ok.values()), ok
    assert r.status_flags & (oracle.QOS_INFEASIBLE | oracle.SIC_INFEASIBLE |
                             oracle.BUDGET_INFEASIBLE) == 0
    assert r.viol_qos == 0.0 and r.viol_budget == 0.0 and r.viol_sic == 0.0
    ev = refeval.evaluate(d, P)
    assert r.ee == pytest.approx(ev["ee"], rel=1e-12)
    # powers are zero or at least 1e-20 of the mask
    pmask = (d.pmax_w / d.N)[:, None, None]
    assert ((r.slot_power == 0) | (r.slot_power >= 1e-20 * pmask)).all()
    np.testing.assert_allclose(r.user_rate, ev["user_rate"], rtol=1e-12, atol=1e-13)
    # the reported association is the RRH whose slots hold the user
    for k in range(d.K):
        holders = [m for m in range(d.M) if (r.sel[m] == k).any()]
        assert len(holders) <= 1
        assert r.rrh_of_user[k] == (holders[0] if holders else -1)
    # sel is in decoding order: normalised gain descending
    tot = P.sum(axis=2)
    G = d.gain.astype(np.float64)
    for m in range(d.M):
        for n in range(d.N):
            us = [k for k in r.sel[m, n] if k >= 0]
            ici = [sum(tot[j, n] * G[j, n, k] for j in range(d.M) if j != m) for k in us]
            gt = [G[m, n, k] / (d.noise_w + i) for k, i in zip(us, ici)]
            assert all(gt[i] >= gt[i + 1] for i in range(len(gt) - 1))


# ------------------------------------------------------------- validation

def test_invalid_inputs_rejected():
    d = synth.make_drop(synth.CFG1, 0, 0)
    bad = synth.make_drop(synth.CFG1, 0, 0)
    bad.l = 0
    with pytest.raises(ValueError):
        oracle.solve(bad)
    bad = synth.make_drop(synth.CFG1, 0, 0)
    bad.l = d.K + 1
    with pytest.raises(ValueError):
        oracle.solve(bad)
    for val in (0.0, -1e-12, np.nan, np.inf):
        g = d.gain.copy()
        g[0, 0, 0] = val
        with pytest.raises(ValueError):
            oracle.solve(d, gain=g)
    bad = synth.make_drop(synth.CFG1, 0, 0)
    bad.delay_s = d.delay_s.copy()
    bad.delay_s[d.user_type == 1] = 0.0
    with pytest.raises(ValueError):
        oracle.solve(bad)


# -------------------------------------------------------------- brute force

def _brute_force(d, psi, levels=17):
    """Global EE optimum over assignments and gridded powers (tiny drops),
    then coordinate refinement of the best grid point."""
    import itertools
    M, N, K, L = d.M, d.N, d.K, d.l
    pmask = d.pmax_w / N
    grid = np.linspace(0.0, 1.0, levels)[1:]
    best = (-1.0, None)
    for A in itertools.product(range(-1, M), repeat=K):
        served = [k for k in range(K) if A[k] >= 0]
        for subsets in itertools.product(range(1, 2 ** N), repeat=len(served)):
            slots = [(A[k], n, k) for k, sub in zip(served, subsets) for n in range(N)
                     if sub >> n & 1]
            cnt = {}
            for (m, n, k) in slots:
                cnt[(m, n)] = cnt.get((m, n), 0) + 1
            if any(c > L for c in cnt.values()):
                continue
            for levs in itertools.product(range(len(grid)), repeat=len(slots)):
                P = np.zeros((M, N, K))
                for (m, n, k), li in zip(slots, levs):
                    P[m, n, k] = grid[li] * pmask[m]
                ok = refeval.feasibility(d, P, L, psi=psi, qos_rel=0.0)
                if not all(ok.values()):
                    continue
                e = refeval.evaluate(d, P)["ee"]
                if e > best[0]:
                    best = (e, P)
    e, P = best
    if P is None:
        return 0.0, None
    # coordinate refinement
    step = 0.5 * (grid[1] - grid[0])
    idx = list(zip(*np.nonzero(P > 0)))
    for _ in range(30):
        for ii in idx:
            for sgn in (+1, -1):
                Q = P.copy()
                Q[ii] = min(max(Q[ii] + sgn * step * pmask[ii[0]], 1e-12), pmask[ii[0]])
                if all(refeval.feasibility(d, Q, L, psi=psi, qos_rel=0.0).values()):
                    e2 = refeval.evaluate(d, Q)["ee"]
                    if e2 > e:
                        e, P = e2, Q
        step *= 0.6
    return e, P


@pytest.mark.slow
def test_brute_force_tiny_instances():
    """On tiny drops: the oracle's allocation meets every constraint (l cap,
    mask, one RRH per user, SIC decodability, budget, and the streaming
    user's minimum rate whenever brute force finds any allocation that meets
    it) and is never better than the global optimum found by brute force.
    The EE ratio to the optimum is reported; the bar on it is soft (the
    method is a local heuristic)."""
    ratios = []
    for seed in range(8):
        rng = np.random.default_rng(500 + seed)
        M, N, K = 2, 2, 2
        gain = 10.0 ** rng.uniform(-13.5, -11.5, (M, N, K))
        ut = [0, 1] if seed % 2 else [0, 0]
        d = custom_drop(gain, user_type=ut, pmax=[2.0, 0.5], eta=[4.0, 2.0], noise=1e-15,
                        l=2, arrival=[0.0, 64e3], delay=[0.0, 0.1])
        psi = psi_of(d)
        r = oracle.solve(d, oracle.Params(fixed_count=0, sweeps_per_dinkelbach=2000))
        P = refeval.dense_from_slots(d, r.sel, r.slot_power)
        ok = refeval.feasibility(d, P, d.l, psi=psi, qos_rel=1e-6, tol=1e-6)
        assert ok["l_cap"] and ok["mask"] and ok["one_rrh"] and ok["sic"] and ok["budget"]
        e_bf, _ = _brute_force(d, psi, levels=9)
        if e_bf > 0:  # a feasible allocation exists on the grid
            assert ok["qos"]
            assert r.ee <= e_bf * (1 + 2e-2)
            ratios.append(r.ee / e_bf)
    ratios = np.array(ratios)
    print("EE / brute-force optimum:", np.round(ratios, 3))
    assert len(ratios) >= 6
    assert np.median(ratios) >= 0.75


def test_oracle_result_independent_of_thread_count():
    """The oracle's sums run in a fixed order: one thread or many give the
    same bits (the benchmark times it both ways)."""
    d = synth.make_drop(synth.CFG2, 3, 0)
    op = oracle.Params(fixed_count=0)
    prev = oracle.set_threads(1)
    try:
        r1 = oracle.solve(d, op)
    finally:
        oracle.set_threads(prev)
    rn = oracle.solve(d, op)
    assert r1.ee == rn.ee and r1.sweeps == rn.sweeps
    np.testing.assert_array_equal(r1.sel, rn.sel)
    np.testing.assert_array_equal(r1.slot_power, rn.slot_power)


# ------------------------------------ streaming users, budget and near-ties

STALL_OFF = dict(CONVERGE, stall_sweeps=0)


def _budget_bound_drop(seed):
    """One RRH, two subcarriers, an elastic and a streaming user, NOMA with
    the spectral mask at the whole budget: the streaming user's power costs
    only the budget multiplier, so the budget binds and its rate settles on
    its minimum."""
    rng = np.random.default_rng(900 + seed)
    gain = 10.0 ** rng.uniform(-12.5, -11.5, (1, 2, 2))
    return custom_drop(gain, user_type=[0, 1], pmax=[0.05], eta=[4.0], noise=1e-15, l=2,
                       arrival=[0.0, 256e3], delay=[0.0, 0.02])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_streaming_kkt_with_binding_budget(seed):
    """KKT at a converged solve with an active minimum rate (C13) and an active
    budget (C12): primal feasibility, complementary slackness
    zeta'(r - Psi) ~ 0 and xi'(pmax - sum p) ~ 0, and stationarity of the
    Lagrangian R - E P + zeta' r_s - xi' sum p in every power (central
    differences)."""
    d = _budget_bound_drop(seed)
    pm = np.array([0.05])
    psi = psi_of(d)
    r = oracle.solve(d, oracle.Params(**STALL_OFF), pmask=pm)
    P = refeval.dense_from_slots(d, r.sel, r.slot_power)
    rs = r.user_rate[1]
    assert rs >= psi[1] * (1 - 1e-6)
    assert r.zeta[1] > 0 and r.xi[0] > 0
    assert abs(r.zeta[1] * (rs / psi[1] - 1.0)) <= 1e-5
    assert abs(r.xi[0] * (P.sum() / d.pmax_w[0] - 1.0)) <= 1e-4
    assert r.status_flags & (oracle.QOS_INFEASIBLE | oracle.BUDGET_INFEASIBLE) == 0
    # the same allocation in a state (a warm start from the dense powers)
    st = oracle.State(d, oracle.Params(**STALL_OFF), warm=dict(p0=P), pmask=pm)
    sel, p, _, _, _ = st.slots()
    E = r.ee

    def lagr(q):
        st.set_powers(q)
        R, Pw, _, ur = st.evaluate()
        return R - E * Pw + r.zeta[1] * ur[1] - r.xi[0] * q[sel >= 0].sum()

    checked = 0
    for idx in zip(*np.nonzero(sel >= 0)):
        h = 1e-6 * p[idx]
        up, dn = p.copy(), p.copy()
        up[idx] += h
        dn[idx] -= h
        grad = (lagr(up) - lagr(dn)) / (2 * h)
        assert abs(grad) <= 1e-5 / (math.log(2) * p[idx]), (idx, grad)
        checked += 1
    assert checked >= 3


def _reachable_drop(seed):
    """A tiny drop whose streaming users can each meet their minimum rate on a
    subcarrier of their own: one RRH (no inter-cell interference), at least
    as many subcarriers as streaming users, and every streaming user's best
    single-subcarrier rate at the mask at least twice its minimum."""
    rng = np.random.default_rng(4000 + seed)
    N = int(rng.integers(2, 5))
    K = int(rng.integers(2, 5))
    ns = int(rng.integers(1, min(N, K - 1) + 1))
    ut = np.zeros(K, np.uint8)
    ut[rng.permutation(K)[:ns]] = 1
    arrival = np.where(ut == 1, rng.uniform(32e3, 256e3, K), 0.0)
    delay = np.where(ut == 1, rng.uniform(0.02, 0.1, K), 0.0)
    gain = 10.0 ** rng.uniform(-13.5, -11.0, (1, N, K))
    d = custom_drop(gain, user_type=ut, pmax=[1.0], eta=[4.0], noise=7e-16,
                    l=int(rng.integers(1, 3)), arrival=arrival, delay=delay)
    psi = psi_of(d)
    best = np.log2(1 + d.gain[0].astype(np.float64).max(axis=0) * (1.0 / N) / d.noise_w)
    return d, psi, bool((best[ut == 1] >= 2 * psi[ut == 1]).all())


def test_minimum_rate_met_whenever_reachable():
    """C13 at the returned allocation: on tiny drops where every streaming
    user can reach twice its minimum rate alone on one subcarrier, the solve
    (default schedule) returns an allocation meeting every minimum rate, and
    C14 holds."""
    done = 0
    for seed in range(80):
        d, psi, reachable = _reachable_drop(seed)
        if not reachable:
            continue
        r = oracle.solve(d, oracle.Params(fixed_count=0))
        s = d.user_type == 1
        assert (r.user_rate[s] >= psi[s] * (1 - 1e-6)).all(), (seed, r.user_rate, psi)
        assert r.status_flags & (oracle.QOS_INFEASIBLE | oracle.SIC_INFEASIBLE) == 0
        done += 1
    assert done >= 40


def test_configuration2_streaming_users_served():
    """On 100 drops of the 5-RRH, 64-subcarrier, 32-user configuration (eight
    streaming users each, minimum rates 0.2-1.6 bits/s/Hz against up to 64
    subcarriers at the mask) no streaming user ends at zero rate, every
    returned allocation meets C12-C14, and the dual loops end on their own
    rules (not all at the sweep cap)."""
    zero = infeasible = 0
    sweeps = []
    for seed in range(100):
        d = synth.make_drop(synth.CFG2, seed, 0)
        r = oracle.solve(d, oracle.Params(fixed_count=0))
        s = d.user_type == 1
        zero += int((r.user_rate[s] <= 0).sum())
        infeasible += bool(r.status_flags & (oracle.QOS_INFEASIBLE | oracle.SIC_INFEASIBLE |
                                              oracle.BUDGET_INFEASIBLE))
        sweeps.append(r.sweeps)
    assert zero == 0
    assert infeasible == 0
    assert sum(x % 200 == 0 for x in sweeps) <= 5


def _tie_drop(delta):
    """One RRH, one subcarrier, two elastic users whose gains differ by the
    relative amount delta, l = 1: the selection compares their H values."""
    gain = np.array([[[1e-12, 1e-12 * (1 + delta)]]])
    return custom_drop(gain, pmax=[0.5], eta=[4.0], noise=1e-15, l=1)


def test_near_tie_flags_at_the_selection():
    """Identical users tie exactly: the (m,n) is flagged and the lower user
    index wins; gains 1e-12 apart (within tie_rel = 1e-9 of each other in H)
    are flagged too; 1e-3 apart they are not, and the stronger user wins."""
    p = oracle.Params(fixed_count=0, sweeps_per_dinkelbach=200)
    for delta, flagged, winner in ((0.0, True, 0), (1e-12, True, None), (1e-3, False, 1)):
        d = _tie_drop(delta)
        r = oracle.solve(d, p, gain=d.gain)
        assert (r.tie_mn[0, 0] > 0) == flagged, (delta, r.tie_mn)
        assert bool(r.status_flags & oracle.NEAR_TIE) == flagged
        if winner is not None:
            assert r.sel[0, 0, 0] == winner
        if not flagged:
            assert r.near_ties == 0


def test_near_tie_flags_at_the_decoding_order():
    """Two users with identical gains sharing a subcarrier (l = 2) have equal
    normalised gains: their decoding order is a near-tie of that (m,n) and
    the lower user index is decoded first."""
    gain = np.full((1, 1, 2), 1e-12)
    d = custom_drop(gain, pmax=[0.5], eta=[4.0], noise=1e-15, l=2)
    r = oracle.solve(d, oracle.Params(fixed_count=0, sweeps_per_dinkelbach=100))
    if (r.sel[0, 0] >= 0).sum() == 2:
        assert r.tie_mn[0, 0] > 0
        assert r.sel[0, 0, 0] == 0
    else:  # one user only: the selection between them is the tie
        assert r.tie_mn[0, 0] > 0 and r.sel[0, 0, 0] == 0


def test_warm_start_from_a_feasible_allocation():
    """A feasible warm allocation is Dinkelbach's p^0 (Sec. III): the first
    step runs no sweeps and sets E^1 = R(p^0)/P(p^0), and the solve never
    returns less than that.  Users go to the RRH of largest total p0 and each
    (m,n) takes its users of largest positive p0, at min(p0, pmask)."""
    d = synth.make_drop(synth.CFG2, 11, 0)
    op = oracle.Params(fixed_count=0)
    cold = oracle.solve(d, op)
    P0 = refeval.dense_from_slots(d, cold.sel, cold.slot_power)
    warm = dict(p0=P0, xi0=cold.xi, zeta0=cold.zeta)
    st = oracle.State(d, op, warm=warm)
    sel, p, xi, zeta, _ = st.slots()
    for m in range(d.M):
        for n in range(d.N):
            assert sorted(k for k in sel[m, n] if k >= 0) == sorted(k for k in cold.sel[m, n] if k >= 0)
    np.testing.assert_array_equal(xi, np.maximum(cold.xi, 0))
    st.close()
    r = oracle.solve(d, op, warm=warm)
    assert r.trace_sweeps[0] == 0
    assert r.trace_E[1] == pytest.approx(cold.ee, rel=1e-12)
    assert r.ee >= cold.ee * (1 - 1e-12)
    assert r.status_flags & oracle.QOS_INFEASIBLE == 0


def test_warm_start_from_an_infeasible_allocation():
    """An infeasible warm allocation (the streaming users given no power) is
    still Dinkelbach's p^0: E^1 = R(p^0)/P(p^0) (the independent evaluator's
    value), which lies above what any feasible allocation reaches here, so
    F < 0 at first and E moves down (F is strictly decreasing in E, Lemma 1).
    The solve ends at the root condition |F| <= tol R on a feasible state
    that meets every minimum rate."""
    d = synth.make_drop(synth.CFG2, 12, 0)
    op = oracle.Params(fixed_count=0)
    cold = oracle.solve(d, op)
    P0 = refeval.dense_from_slots(d, cold.sel, cold.slot_power)
    P0[:, :, d.user_type == 1] = 0.0
    r = oracle.solve(d, op, warm=dict(p0=P0))
    ev = refeval.evaluate(d, P0)
    assert r.trace_sweeps[0] == 0
    assert r.trace_E[1] == pytest.approx(ev["ee"], rel=1e-12)
    assert r.trace_E[1] > cold.ee and r.trace_F[1] < 0
    n = r.dinkelbach_iters
    assert abs(r.trace_F[n - 1]) <= op.tol_dinkelbach * r.trace_R[n - 1]
    assert r.status_flags & (oracle.NOT_CONVERGED | oracle.QOS_INFEASIBLE | oracle.SIC_INFEASIBLE) == 0
    s = d.user_type == 1
    assert (r.user_rate[s] >= psi_of(d)[s] * (1 - 1e-6)).all()


def test_stall_rule_ends_dual_loops_without_progress():
    """The dual loop ends after stall_sweeps sweeps without a better state
    (a violation lower by more than 1e-6 relative counts as better), whether
    or not the best state is feasible, and the next Dinkelbach step restarts
    from the best.  On this drop of the ragged batch generator (3 RRHs, 64
    subcarriers, 216 users, l = 3) no step runs to the sweep cap, the last
    step returns the state it started from (F = 0) after exactly
    stall_sweeps + 1 sweeps, and the result meets C12-C14 (checked by the
    independent evaluator) at Dinkelbach's root condition.  Without the rule
    the first step runs to its cap."""
    d = synth.make_batch(4096, seed=0, indices=[40])[0]
    assert (d.M, d.N, d.K, d.l) == (3, 64, 216, 3)
    op = oracle.Params(fixed_count=0)
    r = oracle.solve(d, op)
    n = r.dinkelbach_iters
    F, sw = r.trace_F[:n], r.trace_sweeps[:n]
    assert (sw < op.sweeps_per_dinkelbach).all(), sw
    assert F[-1] == 0.0 and sw[-1] == op.stall_sweeps + 1, (F, sw)
    assert r.status_flags & (oracle.NOT_CONVERGED | oracle.QOS_INFEASIBLE | oracle.BUDGET_INFEASIBLE
                             | oracle.SIC_INFEASIBLE) == 0
    P = refeval.dense_from_slots(d, r.sel, r.slot_power)
    ok = refeval.feasibility(d, P, d.l, psi=psi_of(d))
    assert all(ok.values()), ok
    assert refeval.sic_violation(d, P) == 0.0
    assert r.ee == pytest.approx(refeval.evaluate(d, P)["ee"], rel=1e-12)
    r0 = oracle.solve(d, oracle.Params(fixed_count=0, stall_sweeps=0, max_dinkelbach=1))
    assert r0.trace_sweeps[0] == op.sweeps_per_dinkelbach


def _sic_broken_state(streaming_weak):
    """Two RRHs, one subcarrier: RRH 0 serves users 0 and 1 together, RRH 1
    serves user 2 at a power whose interference reaches user 0 ten thousand
    times more than user 1.  User 0 has the larger raw gain but, under that
    interference, the smaller normalised gain: the pair breaks C14."""
    gain = np.zeros((2, 1, 3))
    gain[0, 0] = [1e-10, 0.8e-10, 1e-14]
    gain[1, 0] = [1e-9, 1e-13, 1e-10]
    ut = [0, 1 if streaming_weak else 0, 0]
    d = custom_drop(gain, user_type=ut, pmax=[1.0, 1.0], eta=[4.0, 2.0], noise=1e-15, l=2,
                    arrival=[0.0, 64e3, 0.0], delay=[0.0, 0.05, 0.0])
    p0 = np.zeros((2, 1, 3))
    p0[0, 0, 0], p0[0, 0, 1], p0[1, 0, 2] = 0.01, 0.02, 0.1
    return d, p0


@pytest.mark.parametrize("streaming_weak", [True, False])
def test_c14_repair_dissolves_the_breaking_pair(streaming_weak):
    """The repair a solve applies before it returns (C8/C14): the breaking
    pair loses its elastic user when the other is streaming, otherwise the
    user of lower rate (the independent evaluator's rates); the result meets
    C14 and nothing else changes."""
    d, p0 = _sic_broken_state(streaming_weak)
    assert refeval.sic_violation(d, p0) > 0.5
    st = oracle.State(d, oracle.Params(fixed_count=0), warm=dict(p0=p0))
    sel0, p_0, *_ = st.slots()
    assert sorted(sel0[0, 0].tolist()) == [0, 1] and sel0[1, 0, 0] == 2
    rates = refeval.evaluate(d, p0)["user_rate"]
    st.repair_sic()
    sel, p, *_ = st.slots()
    st.close()
    if streaming_weak:
        gone = 0  # the elastic one of (elastic 0, streaming 1)
    else:
        gone = 0 if rates[0] < rates[1] else 1
    kept = 1 - gone
    assert sorted(k for k in sel[0, 0].tolist() if k >= 0) == [kept]
    assert sel[1, 0, 0] == 2 and p[1, 0, 0] == p_0[1, 0, 0]
    P = np.zeros_like(p0)
    P[0, 0, kept], P[1, 0, 2] = p0[0, 0, kept], p0[1, 0, 2]
    assert refeval.sic_violation(d, P) == 0.0


def test_every_output_meets_c14():
    """Drops of the ragged batch generator whose dual loop leaves C14 pairs
    broken, and the 5-RRH configuration: every returned allocation meets
    C12-C14 (the independent evaluator), and EE = R/P of it."""
    drops = synth.make_batch(4096, seed=0, indices=[2061, 40, 1492, 2322, 56])
    drops += [synth.make_drop(synth.CFG2, s, 0) for s in range(4)]
    for d in drops:
        r = oracle.solve(d, oracle.Params(fixed_count=0))
        P = refeval.dense_from_slots(d, r.sel, r.slot_power)
        ok = refeval.feasibility(d, P, d.l, psi=psi_of(d))
        assert all(ok.values()), (d.index, ok)
        assert refeval.sic_violation(d, P) == 0.0 and r.viol_sic == 0.0
        assert r.status_flags & oracle.SIC_INFEASIBLE == 0
        assert r.ee == pytest.approx(refeval.evaluate(d, P)["ee"], rel=1e-12)
