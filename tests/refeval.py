"""Independent numpy evaluation of an allocation (test code only).

Given powers on (RRH, subcarrier, user) triples, computes the SIC-ordered
SINRs, rates, the power model and the energy efficiency of the system model
(Sec. II-A), plus the feasibility of constraints C1-C9 (Sec. II-B).  Written
separately from the oracle so that tests can check its outputs and drive a
brute-force search.
"""
from __future__ import annotations

import numpy as np


def min_rate_quadratic(arrival_bps, delay_s, packet_bits, bw_hz):
    """Psi from the smaller root of the queue-delay quadratic (Sec. II-B)."""
    lam = arrival_bps / packet_bits
    b = 2.0 + 2.0 * lam * delay_s
    root = (b - np.sqrt(b * b - 8.0 * lam * delay_s)) / (2.0 * lam)  # max mean service time
    return packet_bits / (root * bw_hz)


def static_power(drop):
    Mf = drop.M - 1
    return drop.p_fiber_hpn + Mf * drop.p_fiber_lpn + drop.p_circuit_hpn + Mf * drop.p_circuit_lpn


def evaluate(drop, P, weight=None):
    """P: dense powers [M][N][K] (zero = not allocated).

    Returns dict with ee, R, P, user_rate, and per-(m,n) decoding info.
    Decoding on (m,n) by normalised gain Gamma/(sigma+ICI), descending.
    """
    G = drop.gain.astype(np.float64)
    M, N, K = G.shape
    sg = drop.noise_w
    w = np.ones((M, K)) if weight is None else weight
    tot = P.sum(axis=2)  # [M][N]
    rate = np.zeros(K)
    Pel = 0.0
    elastic = drop.user_type == 0
    for m in range(M):
        for n in range(N):
            users = np.nonzero(P[m, n] > 0)[0]
            if users.size == 0:
                continue
            ici = np.array([sum(tot[j, n] * G[j, n, k] for j in range(M) if j != m) for k in users])
            gt = G[m, n, users] / (sg + ici)
            order = sorted(range(users.size), key=lambda i: (-gt[i], users[i]))
            before = 0.0
            for i in order:
                k = users[i]
                I = ici[i] + G[m, n, k] * before
                gam = P[m, n, k] * G[m, n, k] / (sg + I)
                rate[k] += w[m, k] * np.log2(1.0 + gam)
                before += P[m, n, k]
                if elastic[k]:
                    Pel += drop.eta[m] * P[m, n, k]
    R = rate[elastic].sum()
    Ptot = static_power(drop) + Pel
    return dict(ee=R / Ptot, R=R, P=Ptot, user_rate=rate)


def dense_from_slots(drop, sel, slot_power):
    P = np.zeros((drop.M, drop.N, drop.K))
    M, N, L = sel.shape
    for m in range(M):
        for n in range(N):
            for s in range(L):
                k = sel[m, n, s]
                if k >= 0:
                    P[m, n, k] = slot_power[m, n, s]
    return P


def feasibility(drop, P, l, psi=None, pmask=None, qos_rel=1e-6, tol=1e-9):
    """Violations of C1 (l cap), C3/C12 (budget), C4 (mask), C5 (one RRH),
    C8/C14 (SIC) and C9 (QoS).  Returns a dict of booleans (True = holds)."""
    G = drop.gain.astype(np.float64)
    M, N, K = G.shape
    sg = drop.noise_w
    pmask = drop.pmax_w / N if pmask is None else pmask
    ok = {}
    ok["l_cap"] = bool(((P > 0).sum(axis=2) <= l).all())
    ok["budget"] = bool((P.sum(axis=(1, 2)) <= drop.pmax_w * (1 + tol)).all())
    ok["mask"] = bool((P <= pmask[:, None, None] * (1 + tol)).all() and (P >= 0).all())
    served_by = (P.sum(axis=1) > 0)  # [M][K]
    ok["one_rrh"] = bool((served_by.sum(axis=0) <= 1).all())
    tot = P.sum(axis=2)
    sic_ok = True
    for m in range(M):
        for n in range(N):
            users = np.nonzero(P[m, n] > 0)[0]
            for a in range(users.size):
                for b in range(a + 1, users.size):
                    ka, kb = users[a], users[b]
                    s_, w_ = (ka, kb) if G[m, n, ka] >= G[m, n, kb] else (kb, ka)
                    ici = lambda k: sum(tot[j, n] * G[j, n, k] for j in range(M) if j != m)
                    omega = (G[m, n, w_] * sg - G[m, n, s_] * sg + G[m, n, w_] * ici(s_)
                             - G[m, n, s_] * ici(w_))
                    scale = G[m, n, w_] * (sg + ici(s_)) + G[m, n, s_] * (sg + ici(w_))
                    if omega / scale > tol:
                        sic_ok = False
    ok["sic"] = sic_ok
    if psi is not None:
        r = evaluate(drop, P)["user_rate"]
        s = drop.user_type == 1
        ok["qos"] = bool((r[s] >= psi[s] * (1 - qos_rel)).all())
    return ok


def sic_violation(drop, P, tol=1e-9):
    """Sum over co-scheduled pairs of the relative SIC margin Omega/nu (C14,
    scaled by nu = Gamma_w (sigma + ICI_s) + Gamma_s (sigma + ICI_w)) above
    tol; s is the user of larger raw gain (ties to the lower index)."""
    G = drop.gain.astype(np.float64)
    M, N, K = G.shape
    sg = drop.noise_w
    tot = P.sum(axis=2)
    v = 0.0
    for m in range(M):
        for n in range(N):
            users = np.nonzero(P[m, n] > 0)[0]
            if users.size < 2:
                continue
            ici = {k: sum(tot[j, n] * G[j, n, k] for j in range(M) if j != m) for k in users}
            for a in range(users.size):
                for b in range(a + 1, users.size):
                    ka, kb = users[a], users[b]
                    s_, w_ = (ka, kb) if (G[m, n, ka] > G[m, n, kb] or
                                          (G[m, n, ka] == G[m, n, kb] and ka < kb)) else (kb, ka)
                    omega = (G[m, n, w_] * sg - G[m, n, s_] * sg + G[m, n, w_] * ici[s_]
                             - G[m, n, s_] * ici[w_])
                    nu = G[m, n, w_] * (sg + ici[s_]) + G[m, n, s_] * (sg + ici[w_])
                    if omega / nu > tol:
                        v += omega / nu - tol
    return v
