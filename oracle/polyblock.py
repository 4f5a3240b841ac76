"""Global optimum of small drops by monotonic optimization (Sec. IV-B).

TEST INFRASTRUCTURE ONLY: like the rest of ``oracle/`` this module is used by
the tests alone.  It gives the exact optimum (to a stated tolerance) of the
energy-efficiency problem on drops small enough to enumerate, so that the
suboptimal method's optimality gap can be measured.  Plain numpy; nothing here
is shared with the GPU path.

Method.  Dinkelbach's iteration (Sec. III; Theorem 1: E* is the root of the
strictly decreasing F(E) = max_p R(p) - E P(p)) runs around a global solve of
each parametric problem (problem O5 of Sec. IV-B: max R - E P subject to the
mask C4, the selection constraints, the budget C12, the minimum rates C13 and
SIC decodability C14).  The parametric problem is solved exactly in two
layers:

* its discrete part (the RRH of each user, C5/C6, and which of that RRH's
  users may carry power on each subcarrier, at most l of them, C1/C2) is
  enumerated;
* for each such pattern the powers solve a monotonic optimization problem in
  canonical form (Sec. IV-B, Definition of the canonical form: an increasing
  objective over the intersection of a normal and a co-normal set in a
  hyper-rectangle), by the polyblock outer approximation.

Canonical form of one pattern (the rewriting of Sec. IV-B, with one
auxiliary variable per streaming user where the paper folds them into one
with a minimum, and the C14 terms split without the product of the two
powers, since a pattern fixes which pairs share a subcarrier):

* with decoding by raw gain (which C14 makes equal to the decoding by
  normalised gain, Sec. II-A), user k's rate on (m,n) is
  q+_k(p) - q-_k(p), q+ = log2(sigma + ICI_k + Gamma_k * (power of k and the
  users decoded before it)), q- the same without k's own power: both are
  increasing in every power;
* R - E P = Q+(p) - Q-(p) with Q+ = sum over elastic users of w q+ and
  Q- = sum of w q- plus E P(p) (P is increasing in p);
* variables y = (p, s, t_k for streaming k, u_c for each C14 pair that can
  bind), objective f(y) = Q+(p) + s - Q-(b) (b the mask): increasing;
* normal set: p <= b, the budget C12, s + Q-(p) <= Q-(b),
  t_k + q-_k(p) <= q-_k(b), u_c + sum a+_c p <= sum a+_c b;
* co-normal set: q+_k(p) + t_k >= q-_k(b) + Psi_k (C13: at the largest t_k
  the set allows this is r_k >= Psi_k), u_c + sum a-_c p >= sum a+_c b + c0_c
  (C14: Omega = c0 + sum a+ p - sum a- p <= 0 for the pair of users s
  (stronger) and w sharing (m,n), with c0 = sigma (Gamma_w - Gamma_s) and the
  coefficients of the other RRHs' powers on n split by sign).

Polyblock (the four steps listed in Sec. V): the vertex set starts at the
box's upper corner; each iteration takes the vertex of largest objective,
projects it onto the upper boundary of the normal set along the ray from the
origin (bisection), keeps the projection as a feasible point when it lies in
the co-normal set, and replaces the vertex by the d vertices that cut off the
box above the projection; vertices outside the co-normal set (improper: no
feasible point below them), vertices dominated by others and vertices whose
objective cannot beat the best feasible value by more than eps are removed.
The run ends when no vertex can: the best feasible value is then within eps
of the pattern's optimum.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import min_rate


def static_power(d) -> float:
    """P_f^H + M_f P_f^L + P_c^H + M_f P_c^L (Sec. II-A, the power model)."""
    Mf = d.M - 1
    return d.p_fiber_hpn + Mf * d.p_fiber_lpn + d.p_circuit_hpn + Mf * d.p_circuit_lpn


def psi(d) -> np.ndarray:
    """Minimum rate of each streaming user (C9), 0 for elastic users."""
    return np.array([min_rate(a, t, d.packet_bits, d.bw_hz) if ty else 0.0
                     for a, t, ty in zip(d.arrival_bps, d.delay_s, d.user_type)])


class _Pattern:
    """The canonical-form data of one discrete pattern: ``trip`` lists the
    (m, n, k) triples that may carry power."""

    def __init__(self, d, trip, pmask, weight, psi_k, E):
        G = d.gain.astype(np.float64)
        sg = d.noise_w
        nt = len(trip)
        self.trip = trip
        self.nt = nt
        # linear maps: interference at triple i is sigma + p @ Am[:, i]
        # (q-) and sigma + p @ Ap[:, i] (q+)
        Am = np.zeros((nt, nt))
        for i, (m, n, k) in enumerate(trip):
            for j, (m2, n2, k2) in enumerate(trip):
                if n2 != n:
                    continue
                if m2 != m:
                    Am[j, i] = G[m2, n, k]  # other RRHs' power on n reaches k
                elif k2 != k and (G[m, n, k2] > G[m, n, k] or (G[m, n, k2] == G[m, n, k] and k2 < k)):
                    Am[j, i] = G[m, n, k]  # a user decoded before k on (m,n)
        Ap = Am.copy()
        for i, (m, n, k) in enumerate(trip):
            Ap[i, i] = G[m, n, k]
        self.Am, self.Ap, self.sg = Am, Ap, sg
        el = d.user_type == 0
        self.wel = np.array([weight[m, k] if el[k] else 0.0 for (m, n, k) in trip])
        self.eta_el = np.array([d.eta[m] if el[k] else 0.0 for (m, n, k) in trip])
        self.E = E
        self.pstatic = static_power(d)
        self.b = np.array([pmask[m] for (m, n, k) in trip])
        # budget rows (C12)
        self.budget = np.zeros((d.M, nt))
        for i, (m, n, k) in enumerate(trip):
            self.budget[m, i] = 1.0
        self.pmax = np.asarray(d.pmax_w, np.float64)
        # streaming users with power somewhere in the pattern: rate rows
        users = sorted({k for (m, n, k) in trip if not el[k]})
        self.sk = users
        self.U = np.zeros((nt, len(users)))
        for i, (m, n, k) in enumerate(trip):
            if k in users:
                self.U[i, users.index(k)] = weight[m, k]
        self.psi = np.array([psi_k[k] for k in users])
        # C14 pairs that can bind: c0 + a+ p - a- p <= 0
        ap_rows, am_rows, c0s = [], [], []
        for i, (m, n, k) in enumerate(trip):
            for j, (m2, n2, k2) in enumerate(trip):
                if m2 != m or n2 != n or k2 <= k:
                    continue
                s_, w_ = (k, k2) if (G[m, n, k] > G[m, n, k2] or (G[m, n, k] == G[m, n, k2] and k < k2)) else (k2, k)
                a = np.zeros(nt)
                for q, (m3, n3, _) in enumerate(trip):
                    if n3 == n and m3 != m:
                        a[q] = G[m, n, w_] * G[m3, n, s_] - G[m, n, s_] * G[m3, n, w_]
                c0 = sg * (G[m, n, w_] - G[m, n, s_])
                apos, aneg = np.maximum(a, 0.0), np.maximum(-a, 0.0)
                if c0 + apos @ self.b <= 0.0:
                    continue  # holds for every power in the box
                ap_rows.append(apos)
                am_rows.append(aneg)
                c0s.append(c0)
        self.Cp = np.array(ap_rows).reshape(-1, nt)
        self.Cn = np.array(am_rows).reshape(-1, nt)
        self.c0 = np.array(c0s)
        self.ns, self.nc = len(users), len(c0s)
        self.D = nt + 1 + self.ns + self.nc
        # the box of the auxiliary variables
        zero = np.zeros((1, nt))
        bb = self.b[None, :]
        self.Qm_b = self._Qm(bb)[0]
        self.qm_b = self._qm_user(bb)[0]
        self.hi = np.concatenate([
            np.ones(nt),
            [self.Qm_b - self._Qm(zero)[0]],
            self.qm_b - self._qm_user(zero)[0],
            self.Cp @ self.b])
        # power coordinates: p = (sigma / Gamma)(e^(kappa z) - 1), z in [0, 1],
        # kappa = ln(1 + Gamma b / sigma): an increasing map with 0 -> 0, so
        # normal and co-normal sets stay normal and co-normal, and a user's
        # interference-free rate is linear in z (the cuts of the polyblock
        # then act on the rate scale, not the power scale)
        self.gs = np.array([G[m, n, k] for (m, n, k) in trip]) / sg
        self.kappa = np.log1p(self.gs * self.b)

    # -- the increasing functions (rows of P are power vectors)
    def _lm(self, P):
        return np.log2(self.sg + P @ self.Am)

    def _lp(self, P):
        return np.log2(self.sg + P @ self.Ap)

    def _Qm(self, P):
        return self._lm(P) @ self.wel + self.E * (self.pstatic + P @ self.eta_el)

    def _Qp(self, P):
        return self._lp(P) @ self.wel

    def _qm_user(self, P):
        return self._lm(P) @ self.U

    def _qp_user(self, P):
        return self._lp(P) @ self.U

    def powers(self, Z):
        """Powers of the coordinates z (rows)."""
        return np.minimum(np.expm1(self.kappa * Z) / self.gs, self.b)

    def point(self, p):
        """The canonical-form point of powers p (one vector): the auxiliary
        variables at the largest values the normal set allows."""
        P = p[None, :]
        z = np.log1p(self.gs * p) / self.kappa
        t = self.qm_b - self._qm_user(P)[0]
        u = self.Cp @ self.b - self.Cp @ p
        return np.concatenate([z, [self.Qm_b - self._Qm(P)[0]], t, u])[None, :]

    def feasible(self, p):
        """Whether powers p meet the mask, C12, C13 and C14."""
        y = self.point(p)
        return bool(self.in_normal(y, rtol=1e-9)[0] and self.in_conormal(y)[0])

    def split(self, Y):
        nt, ns = self.nt, self.ns
        return self.powers(Y[:, :nt]), Y[:, nt], Y[:, nt + 1:nt + 1 + ns], Y[:, nt + 1 + ns:]

    def f(self, Y):
        P, s, _, _ = self.split(Y)
        return self._Qp(P) + s - self.Qm_b

    def value(self, P):
        """R - E P at powers P (rows)."""
        return self._Qp(P) - self._Qm(P)

    def in_normal(self, Y, rtol=1e-12):
        P, s, t, u = self.split(Y)
        ok = (P <= self.b * (1 + rtol)).all(axis=1)
        ok &= (P @ self.budget.T <= self.pmax * (1 + rtol)).all(axis=1)
        ok &= s + self._Qm(P) <= self.Qm_b + rtol * abs(self.Qm_b)
        if self.ns:
            ok &= (t + self._qm_user(P) <= self.qm_b + rtol * np.abs(self.qm_b)).all(axis=1)
        if self.nc:
            lhs = u + P @ self.Cp.T
            rhs = self.Cp @ self.b
            ok &= (lhs <= rhs * (1 + rtol)).all(axis=1)
        return ok

    def in_conormal(self, Y):
        P, s, t, u = self.split(Y)
        ok = np.ones(len(Y), bool)
        if self.ns:
            ok &= (self._qp_user(P) + t >= self.qm_b + self.psi).all(axis=1)
        if self.nc:
            ok &= (u + P @ self.Cn.T >= self.Cp @ self.b + self.c0).all(axis=1)
        return ok


def polyblock(pat: _Pattern, best: float, eps: float, max_iter: int = 200000, rounds: int = 6):
    """Maximises the pattern's objective over normal ∩ co-normal.  Returns
    (value, powers, upper bound, iterations): the best feasible R - E P found
    above ``best`` (or ``best`` and None), and an upper bound of the pattern's
    optimum (value + eps when the run completed, -inf when the pattern has
    no feasible point)."""
    top = pat.hi[None, :]
    if not pat.in_conormal(top)[0]:
        return best, None, -math.inf, 0
    V = top.copy()
    fV = pat.f(V)
    found = None
    it = 0
    while len(V):
        i = int(np.argmax(fV))
        # every vertex removed so far either had no feasible point below it
        # or could not beat best + eps: the pattern's optimum is at most
        # max(best + eps, the largest objective left)
        if fV[i] <= best + eps:
            return best, found, best + eps, it
        if it >= max_iter:
            return best, found, float(fV[i]), it
        it += 1
        v = V[i]
        if pat.in_normal(v[None, :])[0]:
            lo = hi = 1.0
        else:
            # bisection on the ray, 32 points of it at a time
            lo, hi = 0.0, 1.0
            for _ in range(rounds):
                lam = lo + (hi - lo) * np.arange(1, 33) / 33.0
                inside = pat.in_normal(lam[:, None] * v[None, :])
                j = int(np.argmin(inside)) if not inside.all() else 32
                # the set is normal: the points inside come first
                lo, hi = (lam[j - 1] if j > 0 else lo), (lam[j] if j < 32 else hi)
        x = lo * v
        if pat.in_conormal(x[None, :])[0]:
            px = pat.powers(x[None, :pat.nt])
            val = float(pat.value(px)[0])
            if val > best:
                best, found = val, px[0].copy()
        if hi >= 1.0:  # the vertex itself is feasible: nothing above it is left
            V = np.delete(V, i, axis=0)
            fV = np.delete(fV, i)
            continue
        # replace v by the vertices that cut the box (hi v, v] off
        cut = hi * v
        new = np.repeat(v[None, :], len(v), axis=0)
        idx = np.arange(len(v))
        new[idx, idx] = cut
        keep = v > cut
        new = new[keep]
        V = np.delete(V, i, axis=0)
        fV = np.delete(fV, i)
        if len(new):
            new = new[pat.in_conormal(new)]
        if len(new):
            fn = pat.f(new)
            new, fn = new[fn > best + eps], fn[fn > best + eps]
        if len(new):
            # drop vertices dominated by another vertex
            allv = np.concatenate([V, new])
            nn = len(new)
            dom_new = np.zeros(nn, bool)
            for a in range(nn):
                y = new[a]
                others = np.delete(allv, len(V) + a, axis=0)
                dom_new[a] = bool(((others >= y).all(axis=1)).any())
            new, fn = new[~dom_new], fn[~dom_new]
            if len(new) and len(V):
                dom_old = np.zeros(len(V), bool)
                for a in range(len(new)):
                    dom_old |= (new[a] >= V).all(axis=1)
                V, fV = V[~dom_old], fV[~dom_old]
            V = np.concatenate([V, new])
            fV = np.concatenate([fV, fn])
            del allv
        # prune vertices that cannot beat the new best
        keepv = fV > best + eps
        V, fV = V[keepv], fV[keepv]
    return best, found, best + eps, it


def brb(pat: _Pattern, best: float, eps: float, max_iter: int = 200000, batch: int = 256):
    """Branch-reduce-and-bound over the pattern's power box (the companion of
    the polyblock in the monotonic-optimization framework).  Every slot's rate
    increases in its own power and decreases in the powers that interfere
    with it, and P increases in every power, so on a box [lo, hi] R - E P is
    at most its value with each rate taken at (own power hi, the others lo)
    and P at lo; the box holds no feasible point when the budget fails at
    lo, a minimum rate fails at that bound (C13), or a SIC margin is
    positive with a+ at lo and a- at hi (C14).  Boxes are split in two along the coordinate that contributes
    most to the bound, and dropped once their bound cannot beat the best
    feasible value by more than eps.  Same returns as polyblock()."""
    nt = pat.nt
    b = pat.b

    gain = np.diag(pat.Ap)

    def rates_ub(LO, HI):
        # each slot's rate grows with its own power and falls with every
        # other power that reaches it, so on the box it is at most its value
        # with its own power at hi and the others at lo
        return np.log2(1.0 + gain * HI / (pat.sg + LO @ pat.Am))

    def bound(LO, HI):
        rt = rates_ub(LO, HI)
        ub = rt @ pat.wel - pat.E * (pat.pstatic + LO @ pat.eta_el)
        bad = (LO @ pat.budget.T > pat.pmax * (1 + 1e-12)).any(axis=1)
        if pat.ns:
            bad |= (rt @ pat.U < pat.psi).any(axis=1)
        if pat.nc:
            bad |= (pat.c0 + LO @ pat.Cp.T - HI @ pat.Cn.T > 0.0).any(axis=1)
        return np.where(bad, -np.inf, ub)

    def lower_need(LO, HI, lev):
        # increasing in HI and decreasing in LO: >= 0 wherever a point of
        # the box can reach the level lev and meet C13 and C14
        rt = rates_ub(LO, HI)
        g = rt @ pat.wel - pat.E * (pat.pstatic + LO @ pat.eta_el) - lev
        if pat.ns:
            g = np.minimum(g, (rt @ pat.U - pat.psi).min(axis=1))
        if pat.nc:
            g = np.minimum(g, -(pat.c0 + LO @ pat.Cp.T - HI @ pat.Cn.T).max(axis=1))
        return g

    def upper_need(LO, HI, lev):
        # decreasing in LO: >= 0 wherever the normal constraints and the
        # level can hold
        g = np.minimum(lower_need(LO, HI, lev), (pat.pmax * (1 + 1e-12) - LO @ pat.budget.T).min(axis=1))
        return g

    def reduce(LO, HI, lev, steps=40):
        # the reduction of branch-reduce-and-bound: raise each lower corner
        # coordinate to the least value, and lower each upper one to the
        # largest, at which the box can still hold a point that meets the
        # constraints and beats lev (bisection; both maps are monotone)
        LO, HI = LO.copy(), HI.copy()
        for i in range(nt):
            a, c = LO[:, i].copy(), HI[:, i].copy()
            T = HI.copy()
            T[:, i] = a
            ok = lower_need(LO, T, lev) >= 0
            lo_, hi_ = a.copy(), c.copy()
            for _ in range(steps):
                mid = 0.5 * (lo_ + hi_)
                T[:, i] = mid
                good = lower_need(LO, T, lev) >= 0
                hi_ = np.where(good, mid, hi_)
                lo_ = np.where(good, lo_, mid)
            LO[:, i] = np.where(ok, a, lo_)
        for i in range(nt):
            a, c = LO[:, i].copy(), HI[:, i].copy()
            T = LO.copy()
            T[:, i] = c
            ok = upper_need(T, HI, lev) >= 0
            lo_, hi_ = a.copy(), c.copy()
            for _ in range(steps):
                mid = 0.5 * (lo_ + hi_)
                T[:, i] = mid
                good = upper_need(T, HI, lev) >= 0
                lo_ = np.where(good, mid, lo_)
                hi_ = np.where(good, hi_, mid)
            HI[:, i] = np.where(ok, c, hi_)
        empty = (lower_need(LO, HI, lev) < 0) | (upper_need(LO, HI, lev) < 0) | (LO > HI).any(axis=1)
        return LO, HI, empty

    LO, HI = np.zeros((1, nt)), b[None, :].copy()
    UB = bound(LO, HI)
    if not np.isfinite(UB[0]):
        return best, None, -math.inf, 0
    found = None
    it = 0
    while True:
        live = UB > best + eps
        LO, HI, UB = LO[live], HI[live], UB[live]
        if not len(UB):
            return best, found, best + eps, it
        if it >= max_iter:
            return best, found, float(UB.max()), it
        take = np.argsort(-UB)[:batch]
        lo, hi = LO[take], HI[take]
        it += len(take)
        # feasible points of the boxes: their corners and centres
        for X in (hi, 0.5 * (lo + hi), lo):
            vals = pat.value(X)
            for j in np.argsort(-vals):
                if vals[j] <= best:
                    break
                if pat.feasible(X[j]):
                    best, found = float(vals[j]), X[j].copy()
                    break
        # split each box along the coordinate of largest bound contribution
        contrib = np.empty((len(take), nt))
        base = bound(lo, hi)
        for i in range(nt):
            h2 = hi.copy()
            h2[:, i] = lo[:, i]
            l2 = lo.copy()
            l2[:, i] = hi[:, i]
            contrib[:, i] = np.nan_to_num(2 * base - bound(lo, h2) - bound(l2, hi), neginf=1e300)
        ax = np.argmax(contrib, axis=1)
        r = np.arange(len(take))
        a, c = lo[r, ax], hi[r, ax]
        g = pat.gs[ax]
        # halve the interval on the rate scale while it spans decades of
        # SNR, on the power scale otherwise
        zmid = np.expm1(0.5 * (np.log1p(g * a) + np.log1p(g * c))) / g
        mid = np.where(g * c > 1e3 * (1.0 + g * a), zmid, 0.5 * (a + c))
        lo1, hi1 = lo.copy(), hi.copy()
        hi1[r, ax] = mid
        lo2, hi2 = lo.copy(), hi.copy()
        lo2[r, ax] = mid
        keep = np.ones(len(UB), bool)
        keep[take] = False
        cl, ch = np.concatenate([lo1, lo2]), np.concatenate([hi1, hi2])
        cl, ch, empty = reduce(cl, ch, best + eps)
        cu = np.where(empty, -np.inf, bound(cl, ch))
        LO = np.concatenate([LO[keep], cl])
        HI = np.concatenate([HI[keep], ch])
        UB = np.concatenate([UB[keep], cu])


def patterns(d):
    """Every discrete pattern: each user's RRH (a user with no power is
    listed once, on RRH 0) and, per (m,n), a set of at most l of RRH m's
    users that may carry power (C1/C2, C5/C6)."""
    M, N, K, L = d.M, d.N, d.K, d.l
    for A in itertools.product(range(M), repeat=K):
        per_mn = []
        for m in range(M):
            users = [k for k in range(K) if A[k] == m]
            subs = [c for r in range(min(L, len(users)) + 1) for c in itertools.combinations(users, r)]
            per_mn.extend([subs] * N)
        for choice in itertools.product(*per_mn):
            served = set()
            trip = []
            for idx, sub in enumerate(choice):
                m, n = divmod(idx, N)
                for k in sub:
                    trip.append((m, n, k))
                    served.add(k)
            if any(A[k] != 0 and k not in served for k in range(K)):
                continue  # the same allocation as with the user on RRH 0
            yield tuple(A), trip


def global_optimum(d, pmask=None, weight=None, rel_eps=1e-4, tol_dinkelbach=1e-6, start=None,
                   max_dinkelbach=30, max_iter=200000, method="polyblock"):
    """Globally optimal energy efficiency of drop d (to the stated
    tolerance): Dinkelbach's iteration around the enumerated polyblock
    solves.  ``start``: dense powers [M][N][K] of a feasible allocation whose
    R - E P serves as the first lower bound of each parametric problem (any
    feasible allocation; optional).  Returns a dict:

    * ee_lo: the EE of the best allocation found (a feasible allocation);
    * ee_hi: a certified upper bound of the optimum EE (the last parametric
      problem's upper bound over the static power, added to its E);
    * power: that allocation's dense powers [M][N][K];
    * dinkelbach: parametric problems solved; patterns, iterations: totals.
    """
    M, N, K = d.M, d.N, d.K
    pm = (np.asarray(d.pmax_w, np.float64) / N) if pmask is None else np.asarray(pmask, np.float64)
    w = np.ones((M, K)) if weight is None else np.asarray(weight, np.float64)
    ps = psi(d)
    pats = list(patterns(d))
    E = 0.0
    best_p = None
    n_pat = n_it = 0
    ee_hi = math.inf

    def incumbent(P, E):
        trip = [tuple(x) for x in zip(*np.nonzero(P > 0))]
        if not trip:
            return None
        pat = _Pattern(d, trip, pm, w, ps, E)
        x = np.array([P[t] for t in trip])
        if not pat.feasible(x):
            return None
        return float(pat.value(x[None, :])[0]), (trip, x)

    if start is not None and incumbent(start, 0.0) is not None:
        R0, P0 = _rate_power(d, start, w)
        E = R0 / P0  # F(E) >= 0 at the EE of any feasible allocation
        best_p = start
    for step in range(max_dinkelbach):
        # lower bound of F(E): the incumbent allocation's R - E P
        lb, lb_trip = -math.inf, None
        if best_p is not None:
            got = incumbent(best_p, E)
            if got is not None:
                lb, lb_trip = got
        # the empty allocation is feasible when no user must be served
        if not (d.user_type == 1).any():
            empty = -E * static_power(d)
            if empty > lb:
                lb, lb_trip = empty, ([], np.zeros(0))
        scale = abs(E) * static_power(d) + 1.0
        eps = rel_eps * scale
        ub = lb
        F_best, F_arg = lb, lb_trip
        # a pattern in which no SIC pair can bind allows every one of its
        # triples to carry zero power, so it covers each pattern made of a
        # subset of its triples: those are skipped (largest patterns first)
        covering = []
        for A, trip in sorted(pats, key=lambda x: -len(x[1])):
            if not trip:
                continue
            st = set(trip)
            if any(st <= c for c in covering):
                continue
            n_pat += 1
            pat = _Pattern(d, trip, pm, w, ps, E)
            if pat.nc == 0:
                covering.append(st)
            solver = polyblock if method == "polyblock" else brb
            val, x, up, it = solver(pat, F_best, eps, max_iter=max_iter)
            n_it += it
            ub = max(ub, up)
            if x is not None and val > F_best:
                F_best, F_arg = val, (trip, x)
        if F_arg is None:
            return dict(ee_lo=0.0, ee_hi=0.0, power=None, dinkelbach=step + 1, patterns=n_pat,
                        iterations=n_it, feasible=False)
        trip, x = F_arg
        P = np.zeros((M, N, K))
        for t, v in zip(trip, x):
            P[t] = v
        best_p = P
        # F(E) <= ub, and F(E*) = 0 with P >= static power:
        # E* <= E + F(E) / P_static
        ee_hi = E + max(ub, 0.0) / static_power(d)
        R, Ptot = _rate_power(d, P, w)
        E_new = R / Ptot
        # F(E) <= ub: stop once F(E) is within the tolerance of zero, or E
        # no longer moves
        if ub <= max(tol_dinkelbach * R, 2 * eps) or E_new <= E * (1 + 1e-12):
            E = max(E, E_new)
            break
        E = E_new
    return dict(ee_lo=E, ee_hi=max(ee_hi, E), power=best_p, dinkelbach=step + 1, patterns=n_pat,
                iterations=n_it, feasible=True)


def _rate_power(d, P, w):
    """R and P (Sec. II-A) of dense powers with decoding by raw gain."""
    G = d.gain.astype(np.float64)
    M, N, K = G.shape
    sg = d.noise_w
    tot = P.sum(axis=2)
    R = 0.0
    Pel = 0.0
    for m in range(M):
        for n in range(N):
            users = [k for k in range(K) if P[m, n, k] > 0]
            for k in users:
                ici = sum(tot[j, n] * G[j, n, k] for j in range(M) if j != m)
                before = sum(P[m, n, j] for j in users
                             if G[m, n, j] > G[m, n, k] or (G[m, n, j] == G[m, n, k] and j < k))
                r = w[m, k] * math.log2(1.0 + P[m, n, k] * G[m, n, k] / (sg + ici + G[m, n, k] * before))
                if d.user_type[k] == 0:
                    R += r
                    Pel += d.eta[m] * P[m, n, k]
    return R, static_power(d) + Pel
