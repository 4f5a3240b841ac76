"""Comparison of a GPU result with the FP64 oracle's (test code).

Bars (the measurement target): EE within 1e-5 relative; every power within
1e-4 relative above a floor of 1e-6 * pmask (absolute below it); identical
association and selection, and identical Dinkelbach/sweep counts, unless the
oracle flags a near-tie.  User rates follow from the powers: a 1e-4 relative
power change moves a rate by at most 1e-4/ln 2 per slot, so rates are compared
at rtol 1e-4 with an absolute 2e-4.

Some drops are rounding-chaotic: the method itself (discrete selection,
projections at zero) amplifies differences of one ulp.  When a strict check
fails, the oracle is re-run with the noise power moved by a few ulps; if the
oracle's own result then breaks the same check at least as badly, the drop is
marked chaotic and only the EE bar and the structural checks apply.  Callers
count chaotic drops and bound their share.
"""
from __future__ import annotations

import numpy as np

EE_RTOL = 1e-5
P_RTOL = 1e-4
P_FLOOR = 1e-6
RATE_RTOL = 1e-4
RATE_ATOL = 2e-4
MULT_RTOL = 1e-6
MULT_ATOL = 1e-9


def _discrepancies(drop, a, b, pm):
    """Named violations between two results (a compared to reference b)."""
    out = {}
    if a.dinkelbach_iters != b.dinkelbach_iters or a.sweeps != b.sweeps:
        out["counts"] = 1.0
    if not np.array_equal(a.rrh_of_user, b.rrh_of_user):
        out["assoc"] = float((a.rrh_of_user != b.rrh_of_user).sum())
    if not np.array_equal(a.sel, b.sel):
        out["sel"] = float((a.sel != b.sel).sum())
        return out
    floor = np.broadcast_to((P_FLOOR * pm)[:, None, None], b.slot_power.shape)
    big = np.abs(b.slot_power) > floor
    rel = np.abs(a.slot_power - b.slot_power) / np.maximum(np.abs(b.slot_power), 1e-300)
    prel = float(rel[big].max()) if big.any() else 0.0
    if prel > P_RTOL:
        out["power"] = prel
    small_bad = np.abs(a.slot_power - b.slot_power)[~big] > floor[~big]
    if small_bad.any():
        out["power_small"] = float(small_bad.sum())
    dr = np.abs(a.user_rate - b.user_rate) - (RATE_ATOL + RATE_RTOL * np.abs(b.user_rate))
    if (dr > 0).any():
        out["rate"] = float(np.abs(a.user_rate - b.user_rate).max())
    for name in ("xi", "zeta", "zeta_sic"):
        x, y = getattr(a, name), getattr(b, name)
        bad = np.abs(x - y) - (MULT_ATOL + MULT_RTOL * np.abs(y))
        if (bad > 0).any():
            out[name] = float(np.abs(x - y).max())
    return out


def compare(drop, gpu, orc, pmask=None, label="", rerun=None):
    """Raises AssertionError on a violation; returns a dict of measurements.

    ``rerun(noise_scale)`` re-solves the drop with the oracle at a scaled
    noise power (used only when a strict check fails)."""
    pm = (drop.pmax_w / drop.N) if pmask is None else np.asarray(pmask, dtype=np.float64)
    info = dict(label=label, near_ties=int(orc.near_ties))
    assert gpu.sel.shape == orc.sel.shape
    info["ee_rel"] = abs(gpu.ee - orc.ee) / max(abs(orc.ee), 1e-300)
    if orc.near_ties > 0:
        info["skipped"] = "near-tie"
        return info
    assert info["ee_rel"] <= EE_RTOL, info
    bad = _discrepancies(drop, gpu, orc, pm)
    info["violations"] = bad
    if not bad:
        return info
    assert rerun is not None, info
    worst = {}
    for scale in (1.0 + 2.0 ** -50, 1.0 - 2.0 ** -50, 1.0 + 2.0 ** -48):
        alt = rerun(scale)
        own = _discrepancies(drop, alt, orc, pm)
        for k, v in own.items():
            worst[k] = max(worst.get(k, 0.0), v)
    info["oracle_self"] = worst
    for k, v in bad.items():
        assert k in worst and worst[k] >= 0.1 * v, info
    info["skipped"] = "chaotic"
    # what stays unique: sizes and the structural checks
    return info
