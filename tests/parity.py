"""Comparison of a GPU result with the FP64 oracle's (test code).

Bars (the measurement target): EE within 1e-5 relative; every power within
1e-4 relative above a floor of 1e-6 * pmask (absolute below it); identical
association, selection and decoding order, and identical Dinkelbach/sweep
counts and status flags.  User rates follow from the powers: a 1e-4 relative
power change moves a rate by at most 1e-4/ln 2 per slot, so rates are
compared at rtol 1e-4 with an absolute 2e-4.  Multipliers at 1e-6 relative.

Near-ties.  Both sides compute in FP64, with different summation orders, so
a discrete decision whose relative margin is within a few ulps may go either
way.  The oracle counts every decision whose margin is below tie_rel and
records which (RRH, subcarrier) pairs and which users they concern
(tie_mn, tie_user).  Then:

* the EE bar always applies;
* the selection, decoding order and powers of every unflagged (m,n), and the
  association of every unflagged user, are compared at the bars above;
* counts, flags, rates and multipliers, which depend on every decision, are
  compared when the oracle flagged nothing;
* a drop whose flagged decision went the other way and moved the trajectory
  (unflagged elements differ) fails, unless the caller allows it
  (``allow_diverged``): then the EE bar becomes EE_RTOL_DIVERGED and the
  result must be a valid allocation.  Callers bound such drops.
"""
from __future__ import annotations

import numpy as np

EE_RTOL = 1e-5
EE_RTOL_DIVERGED = 1e-2
P_RTOL = 1e-4
P_FLOOR = 1e-6
RATE_RTOL = 1e-4
RATE_ATOL = 2e-4
MULT_RTOL = 1e-6
MULT_ATOL = 1e-9


def _flags(orc, name, shape):
    v = getattr(orc, name, None)
    return np.zeros(shape, bool) if v is None else np.asarray(v) > 0


def _discrepancies(drop, a, b, pm, tmn, tu, strict):
    """Named violations between result a and reference b on the elements not
    flagged (tmn [M][N], tu [K]); strict adds the whole-solve quantities."""
    out = {}
    keep_mn = ~tmn
    assoc = (a.rrh_of_user != b.rrh_of_user) & ~tu
    if assoc.any():
        out["assoc"] = float(assoc.sum())
    seld = (a.sel != b.sel).any(axis=2) & keep_mn
    if seld.any():
        out["sel"] = float(seld.sum())
    same = keep_mn & ~(a.sel != b.sel).any(axis=2)
    floor = np.broadcast_to((P_FLOOR * pm)[:, None, None], b.slot_power.shape)
    big = (np.abs(b.slot_power) > floor) & same[:, :, None]
    small = (np.abs(b.slot_power) <= floor) & same[:, :, None]
    rel = np.abs(a.slot_power - b.slot_power) / np.maximum(np.abs(b.slot_power), 1e-300)
    prel = float(rel[big].max()) if big.any() else 0.0
    if prel > P_RTOL:
        out["power"] = prel
    small_bad = np.abs(a.slot_power - b.slot_power)[small] > floor[small]
    if small_bad.any():
        out["power_small"] = float(small_bad.sum())
    if b.zeta_sic.size:
        zs = np.abs(a.zeta_sic - b.zeta_sic) - (MULT_ATOL + MULT_RTOL * np.abs(b.zeta_sic))
        zbad = (zs > 0).any(axis=2) & same
        if zbad.any():
            out["zeta_sic"] = float(zbad.sum())
    if not strict:
        return out
    if a.dinkelbach_iters != b.dinkelbach_iters or a.sweeps != b.sweeps:
        out["counts"] = 1.0
    fa, fb = int(a.status_flags) & ~4, int(b.status_flags) & ~4  # NEAR_TIE is the oracle's
    if fa != fb:
        out["flags"] = float(fa ^ fb)
    dr = np.abs(a.user_rate - b.user_rate) - (RATE_ATOL + RATE_RTOL * np.abs(b.user_rate))
    if (dr > 0).any():
        out["rate"] = float(np.abs(a.user_rate - b.user_rate).max())
    for name in ("xi", "zeta"):
        x, y = getattr(a, name), getattr(b, name)
        bad = np.abs(x - y) - (MULT_ATOL + MULT_RTOL * np.abs(y))
        if (bad > 0).any():
            out[name] = float(np.abs(x - y).max())
    return out


def check_structure(drop, r, pmask=None):
    """What holds for any allocation the solver returns: at most l distinct
    users per (m,n), each user on one RRH (C5/C6) as rrh_of_user says, powers
    within the mask and zero on empty slots, EE = rate / power."""
    sel, sp = r.sel, r.slot_power
    assert sel.shape == (drop.M, drop.N, drop.l)
    assert ((sel >= -1) & (sel < drop.K)).all()
    mask = drop.pmax_w / drop.N if pmask is None else np.asarray(pmask, np.float64)
    assert (sp >= 0).all() and (sp <= mask[:, None, None] * (1 + 1e-12)).all()
    assert (sp[sel < 0] == 0).all()
    served_by = np.full(drop.K, -1)
    for m in range(drop.M):
        for n in range(drop.N):
            users = sel[m, n][sel[m, n] >= 0]
            assert len(set(users.tolist())) == len(users)
            assert ((served_by[users] == -1) | (served_by[users] == m)).all()
            served_by[users] = m
    assert np.array_equal(served_by, r.rrh_of_user)
    assert np.isfinite(r.ee)
    if r.power_sum > 0:
        assert abs(r.ee - r.rate_sum / r.power_sum) <= 1e-12 * max(abs(r.ee), 1e-300)


def compare(drop, gpu, orc, pmask=None, label="", allow_diverged=False):
    """Raises AssertionError on a violation; returns a dict of measurements
    (flagged: the oracle's flagged (m,n) pairs and users; diverged: a flagged
    decision moved the trajectory)."""
    pm = (drop.pmax_w / drop.N) if pmask is None else np.asarray(pmask, dtype=np.float64)
    assert gpu.sel.shape == orc.sel.shape
    tmn = _flags(orc, "tie_mn", (drop.M, drop.N))
    tu = _flags(orc, "tie_user", (drop.K,))
    ties = int(orc.near_ties)
    info = dict(label=label, near_ties=ties, flagged_mn=int(tmn.sum()), flagged_users=int(tu.sum()))
    info["ee_rel"] = abs(gpu.ee - orc.ee) / max(abs(orc.ee), 1e-300)
    bad = _discrepancies(drop, gpu, orc, pm, tmn, tu, strict=ties == 0)
    info["violations"] = bad
    if not bad or ties == 0:
        assert info["ee_rel"] <= EE_RTOL and not bad, info
        return info
    # a flagged decision went the other way and moved the trajectory
    info["diverged"] = True
    assert allow_diverged, info
    assert info["ee_rel"] <= EE_RTOL_DIVERGED, info
    check_structure(drop, gpu, pmask)
    return info


class Stored:
    """An oracle result read back from a stored .npz (tests/golden)."""


def load_stored(g, prefix, drop):
    """The stored oracle result of ``drop`` under ``prefix`` in the loaded
    archive g (as tests/golden/make_cfg4_goldens.py writes it); checks that
    the drop's gains are the ones the oracle solved."""
    import hashlib
    if hashlib.sha256(drop.gain.tobytes()).digest() != g[prefix + "gain_sha256"].tobytes():
        raise ValueError(f"{prefix}: gains differ from the stored oracle run")
    o = Stored()
    o.sel = g[prefix + "sel"].astype(np.int32)
    o.slot_power = g[prefix + "slot_power"].astype(np.float64)
    o.rrh_of_user = g[prefix + "rrh_of_user"].astype(np.int32)
    o.user_rate, o.xi, o.zeta = g[prefix + "user_rate"], g[prefix + "xi"], g[prefix + "zeta"]
    o.zeta_sic = np.zeros((drop.M, drop.N, 0))
    o.tie_mn, o.tie_user = g[prefix + "tie_mn"], g[prefix + "tie_user"]
    o.ee, o.rate_sum, o.power_sum, o.viol_qos, o.viol_budget, o.viol_sic = (
        float(x) for x in g[prefix + "scalars"])
    o.dinkelbach_iters, o.sweeps, o.status_flags, o.near_ties = (int(x) for x in g[prefix + "ints"])
    return o
