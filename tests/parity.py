"""Comparison of a GPU result with the FP64 oracle's (test code)."""
from __future__ import annotations

import numpy as np

# Tolerances of the measurement target: EE 1e-5 relative, each power 1e-4
# relative above a floor of 1e-6 * pmask, identical discrete decisions unless
# the oracle flags a near-tie.
EE_RTOL = 1e-5
P_RTOL = 1e-4
P_FLOOR = 1e-6


def compare(drop, gpu, orc, pmask=None, label=""):
    """Returns a dict of measured differences; raises AssertionError on a
    violation.  Drops whose oracle trajectory has a near-tie are only checked
    for what is unique (sizes, flags other than ties)."""
    pm = (drop.pmax_w / drop.N) if pmask is None else np.asarray(pmask)
    info = dict(label=label, near_ties=int(orc.near_ties))
    assert gpu.sel.shape == orc.sel.shape
    if orc.near_ties > 0:
        info["skipped"] = True
        return info
    info["ee_rel"] = abs(gpu.ee - orc.ee) / max(abs(orc.ee), 1e-300)
    assert info["ee_rel"] <= EE_RTOL, info
    assert gpu.dinkelbach_iters == orc.dinkelbach_iters, (gpu.dinkelbach_iters, orc.dinkelbach_iters)
    assert gpu.sweeps == orc.sweeps, (gpu.sweeps, orc.sweeps)
    assert np.array_equal(gpu.rrh_of_user, orc.rrh_of_user), label
    assert np.array_equal(gpu.sel, orc.sel), label
    floor = (P_FLOOR * pm)[:, None, None]
    big = np.abs(orc.slot_power) > floor
    rel = np.abs(gpu.slot_power - orc.slot_power) / np.maximum(np.abs(orc.slot_power), 1e-300)
    info["p_rel_max"] = float(rel[big].max()) if big.any() else 0.0
    assert info["p_rel_max"] <= P_RTOL, info
    assert (np.abs(gpu.slot_power - orc.slot_power)[~big] <= floor.repeat(drop.N, 1).repeat(drop.l, 2)[~big]).all()
    np.testing.assert_allclose(gpu.user_rate, orc.user_rate, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(gpu.xi, orc.xi, rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(gpu.zeta, orc.zeta, rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(gpu.zeta_sic, orc.zeta_sic, rtol=1e-6, atol=1e-9)
    assert (gpu.status_flags & ~4) == (orc.status_flags & ~4)
    info["rate_rel"] = float(np.max(np.abs(gpu.user_rate - orc.user_rate) /
                                    np.maximum(np.abs(orc.user_rate), 1e-12)))
    return info
