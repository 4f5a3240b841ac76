"""The paper's own relaxation of the selection constraints (Sec. II-B, C10 and
C11; Sec. IV-A, the multipliers theta and theta') on small drops.

TEST INFRASTRUCTURE ONLY: like the rest of ``oracle/`` this module is used by
the tests alone.  It cross-checks the reading the oracle and the GPU path take
for the binary constraints (an exact selection of at most l users per (m,n)
and one RRH per user, chosen by the per-triple Lagrangian maximum) against the
paper's literal relaxation, in which every (RRH, subcarrier, user) triple
carries a power and the binary constraints become product constraints:

* C10: for every user and every two triples of it on different RRHs, the
  product of the two powers is at most rho1 (so a user keeps significant
  power on one RRH only);
* C11: on every (m,n), the product of the powers of any l + 1 distinct users
  is at most rho2 (the paper writes it for l = 3: four users).

Both are written on powers relative to the mask, (p/pmask)(p'/pmask') <=
rho1 and prod (p/pmask) <= rho2, so that rho is scale-free.  Their
multipliers enter the closed-form powers as extra prices in the denominator:
the derivative of theta * prod with respect to the power (Sec. IV-A,
eq. of the elastic and streaming powers, the terms with theta and theta').
Their subgradient steps use the violation relative to rho (the C13 step of
the method does the same with Psi), bounded below by -1 and not above: a
multiplier has to reach about 1/rho before it drives a product down to rho.

Everything else is the method as the oracle implements it (Sec. IV-A,
Alg. 1): SIC-ordered SINRs by normalised gain, the SCALE refit, the full
gradient prices over all victims, the budget multiplier xi' and the
minimum-rate multiplier zeta', Jacobi sweeps inside Dinkelbach steps.  The
C14 multipliers are left out: the drops this is meant for have one RRH
(no inter-cell interference, so every pair decodes in raw-gain order) or
l = 1 (no pair survives).  Plain numpy loops: drops of a few RRHs,
subcarriers and users only.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import min_rate

LN2 = math.log(2.0)


def _static_power(d) -> float:
    Mf = d.M - 1
    return d.p_fiber_hpn + Mf * d.p_fiber_lpn + d.p_circuit_hpn + Mf * d.p_circuit_lpn


def solve_relaxed(d, rho1: float, rho2: float, max_dinkelbach: int = 30, sweeps: int = 4000,
                  tol_dual: float = 1e-9, tol_dinkelbach: float = 1e-7, step0: float = 0.1,
                  qos_down: float = 0.2, weight=None, p0=None):
    """Dinkelbach + SCALE + dual with the C10/C11 product constraints on
    every triple, from powers p0 [M][N][K] (clipped to the mask), else from
    an equal share of the mask on every triple.  Returns a dict: p [M][N][K]
    powers, ee, rate_sum, power_sum, user_rate [K], and the worst normalised
    C10/C11 products."""
    M, N, K, L = d.M, d.N, d.K, d.l
    G = d.gain.astype(np.float64)
    sg = d.noise_w
    pm = np.asarray(d.pmax_w, np.float64) / N
    pmax = np.asarray(d.pmax_w, np.float64)
    eta = np.asarray(d.eta, np.float64)
    w = np.ones((M, K)) if weight is None else np.asarray(weight, np.float64)
    el = d.user_type == 0
    psi = np.array([min_rate(a, t, d.packet_bits, d.bw_hz) if ty else 0.0
                    for a, t, ty in zip(d.arrival_bps, d.delay_s, d.user_type)])
    pstatic = _static_power(d)
    # C10 pairs: (m, n, m2, n2) with m < m2, per user; C11 sets: (m, n, S)
    c10 = [(m, n, m2, n2) for m in range(M) for m2 in range(m + 1, M) for n in range(N) for n2 in range(N)]
    c11 = [(m, n, S) for m in range(M) for n in range(N) for S in itertools.combinations(range(K), L + 1)]
    th = np.zeros((len(c10), K))
    th2 = np.zeros(len(c11))
    # start: every triple at an equal share of the mask
    p = np.repeat((pm / K)[:, None, None], N, axis=1).repeat(K, axis=2)
    if p0 is not None:
        p = np.minimum(np.maximum(np.asarray(p0, np.float64), 0.0), pm[:, None, None])
    al = np.ones((M, N, K))
    be = np.zeros((M, N, K))
    xi = np.zeros(M)
    zeta = np.where(el, 0.0, 1.0)
    E = 0.0
    v = 0

    def evaluate(p, al, be, refit):
        """SINRs, rates and surrogate rates, price weights; refits alpha and
        beta where asked (Sec. IV-A)."""
        tot = p.sum(axis=2)
        ici = np.zeros((M, N, K))
        for m in range(M):
            for n in range(N):
                ici[m, n] = sum(tot[j, n] * G[j, n] for j in range(M) if j != m)
        rate = np.zeros((M, N, K))
        rhat = np.zeros((M, N, K))
        cw = np.zeros((M, N, K))  # c_v = w mu alpha / (ln2 (sigma + I_v))
        after = np.zeros((M, N, K))  # sum of c_v Gamma_v over users decoded after k
        al, be = al.copy(), be.copy()
        for m in range(M):
            for n in range(N):
                users = [k for k in range(K) if p[m, n, k] > 0.0]
                gt = {k: G[m, n, k] / (sg + ici[m, n, k]) for k in users}
                order = sorted(users, key=lambda k: (-gt[k], k))
                before = 0.0
                for k in order:
                    I = ici[m, n, k] + G[m, n, k] * before
                    gam = p[m, n, k] * G[m, n, k] / (sg + I)
                    if refit:
                        al[m, n, k] = gam / (1.0 + gam)
                        be[m, n, k] = math.log2(1.0 + gam) - al[m, n, k] * math.log2(gam)
                    rate[m, n, k] = math.log2(1.0 + gam)
                    rhat[m, n, k] = be[m, n, k] + al[m, n, k] * math.log2(gam)
                    mu = 1.0 if el[k] else zeta[k]
                    cw[m, n, k] = w[m, k] * mu * al[m, n, k] / (LN2 * (sg + I))
                    before += p[m, n, k]
                acc = 0.0
                for k in reversed(order):
                    after[m, n, k] = acc
                    acc += cw[m, n, k] * G[m, n, k]
        return ici, rate, rhat, cw, after, al, be

    def totals(p, rate):
        R = float((rate.sum(axis=1)[:, el] * w[:, el]).sum())
        P = pstatic + float((eta[:, None] * p[:, :, el].sum(axis=1)).sum())
        return R, P

    trace = []
    for _ in range(max_dinkelbach):
        al[:] = 1.0
        be[:] = 0.0
        for s in range(sweeps):
            ici, rate, rhat, cw, after, al, be = evaluate(p, al, be, refit=True)
            # inter-cell price of triple (m,n,k): what its power costs the
            # users of the other RRHs on n
            inter = np.zeros((M, N))
            for m in range(M):
                for n in range(N):
                    inter[m, n] = sum(cw[j, n, u] * G[m, n, u] for j in range(M) if j != m for u in range(K))
            # the relaxation's prices: derivative of theta * product
            pr10 = np.zeros((M, N, K))
            for c, (m, n, m2, n2) in enumerate(c10):
                pr10[m, n] += th[c] * p[m2, n2] / (pm[m] * pm[m2])
                pr10[m2, n2] += th[c] * p[m, n] / (pm[m] * pm[m2])
            pr11 = np.zeros((M, N, K))
            for c, (m, n, S) in enumerate(c11):
                for k in S:
                    others = [u for u in S if u != k]
                    pr11[m, n, k] += th2[c] * np.prod(p[m, n, others] / pm[m]) / pm[m]
            pn = np.zeros_like(p)
            for m in range(M):
                for n in range(N):
                    for k in range(K):
                        mu = 1.0 if el[k] else zeta[k]
                        num = w[m, k] * mu * al[m, n, k] / LN2
                        den = (E * eta[m] if el[k] else 0.0) + xi[m] + after[m, n, k] + inter[m, n] \
                            + pr10[m, n, k] + pr11[m, n, k]
                        q = num / den if den > 0.0 else pm[m]
                        q = min(max(q, 0.0), pm[m])
                        # powers below 1e-20 of the mask are zero, as in the
                        # method (a decaying power would underflow the SINR)
                        pn[m, n, k] = q if q >= 1e-20 * pm[m] else 0.0
            delta = step0 / math.sqrt(1.0 + v)
            v += 1
            dmax = float((np.abs(pn - p) / pm[:, None, None]).max())
            # subgradient steps (Sec. IV-A, Alg. 1): budget, minimum rates,
            # and the product constraints relative to rho
            xi = np.maximum(xi + delta * N * L / (LN2 * pmax) * (pn.sum(axis=(1, 2)) - pmax) / pmax, 0.0)
            rk = (rhat * w[:, None, :]).sum(axis=(0, 1))
            for k in range(K):
                if not el[k]:
                    g = min(max((psi[k] - rk[k]) / psi[k], -qos_down), 1.0)
                    zeta[k] = max(zeta[k] + delta * g, 0.0)
            for c, (m, n, m2, n2) in enumerate(c10):
                x = pn[m, n] * pn[m2, n2] / (pm[m] * pm[m2])
                th[c] = np.maximum(th[c] + delta * np.maximum((x - rho1) / rho1, -1.0), 0.0)
            for c, (m, n, S) in enumerate(c11):
                x = float(np.prod(pn[m, n, list(S)] / pm[m]))
                th2[c] = max(th2[c] + delta * max((x - rho2) / rho2, -1.0), 0.0)
            p = pn
            if dmax < tol_dual:
                break
        _, rate, _, _, _, _, _ = evaluate(p, al, be, refit=False)
        R, P = totals(p, rate)
        F = R - E * P
        trace.append((E, F, s + 1))
        if abs(F) <= tol_dinkelbach * max(R, 1e-300):
            break
        E = R / P
    _, rate, _, _, _, _, _ = evaluate(p, al, be, refit=False)
    R, P = totals(p, rate)
    x10 = max((float((p[m, n] * p[m2, n2] / (pm[m] * pm[m2])).max()) for (m, n, m2, n2) in c10), default=0.0)
    x11 = max((float(np.prod(p[m, n, list(S)] / pm[m])) for (m, n, S) in c11), default=0.0)
    return dict(p=p, ee=R / P, rate_sum=R, power_sum=P, user_rate=(rate * w[:, None, :]).sum(axis=(0, 1)),
                c10_max=x10, c11_max=x11, trace=trace, sweeps=v)
