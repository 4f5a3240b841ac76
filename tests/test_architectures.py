"""The architecture variants of the paper's simulation section (Sec. VIII,
the comparison of H-CRAN with C-RAN, HCN and 1-tier HPN, and of PD-NOMA with
OMA): how the inputs are built, and that the oracle charges each network its
own power model (Sec. II-A: static power of every site plus each site's
transmit power times its power-efficiency factor eta)."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

# static power of each site (circuit + fronthaul) per architecture, from the
# paper's simulation settings: HPN 3 + 3 W, LPN 0.1 + 1 W; macro BS 10 W,
# pico BS 6.8 W, no fronthaul
SITE_STATIC = {
    "hcran": [6.0, 1.1, 1.1],
    "oma": [6.0, 1.1, 1.1],
    "cran": [1.1, 1.1, 1.1],
    "hcn": [10.0, 6.8, 6.8],
    "hpn": [10.0, 10.0],
}
SITE_ETA = {"hcran": [4, 2, 2], "oma": [4, 2, 2], "cran": [2, 2, 2], "hcn": [4, 4, 4], "hpn": [4, 4]}
HPN_W, LPN_W = 10 ** (42 / 10) / 1e3, 10 ** (23 / 10) / 1e3
SITE_PMAX = {"hcran": [HPN_W, LPN_W, LPN_W], "oma": [HPN_W, LPN_W, LPN_W], "cran": [LPN_W] * 3,
             "hcn": [HPN_W, LPN_W, LPN_W], "hpn": [HPN_W, HPN_W]}


def _solver_static(d):
    """The static power the solver charges: RRH 0 the hpn terms, the rest the lpn ones."""
    return d.p_fiber_hpn + d.p_circuit_hpn + (d.M - 1) * (d.p_fiber_lpn + d.p_circuit_lpn)


@pytest.mark.parametrize("arch", synth.ARCHITECTURES)
def test_architecture_inputs(arch):
    base = synth.architecture_drop("hcran", 3, 7)
    d = synth.architecture_drop(arch, 3, 7)
    M = len(SITE_STATIC[arch])
    assert d.M == M and d.gain.shape == (M, d.N, d.K) and d.l == (1 if arch == "oma" else base.l)
    assert _solver_static(d) == pytest.approx(sum(SITE_STATIC[arch]), rel=1e-12)
    np.testing.assert_allclose(d.eta, SITE_ETA[arch])
    np.testing.assert_allclose(d.pmax_w, SITE_PMAX[arch], rtol=1e-12)
    # same users and fading on the sites it keeps
    np.testing.assert_array_equal(d.gain, base.gain[:M])
    np.testing.assert_array_equal(d.user_type, base.user_type)
    np.testing.assert_array_equal(d.arrival_bps, base.arrival_bps)
    np.testing.assert_array_equal(d.user_xy, base.user_xy)


def test_architectures_need_the_paper_channel():
    with pytest.raises(ValueError):
        synth.architecture_drop("hcn", 0, 0, recipe=synth.CFG2)
    with pytest.raises(ValueError):
        synth.architecture_drop("femto", 0, 0)


@pytest.mark.parametrize("arch", synth.ARCHITECTURES)
def test_oracle_power_model_per_architecture(arch):
    """The objective's power: the sum of the site static powers plus
    sum_m eta_m (m's power to elastic users); its rate: the elastic users'
    rates; EE their ratio, with each architecture's own constants."""
    d = synth.architecture_drop(arch, 1, 2)
    r = oracle.solve(d, oracle.Params(fixed_count=0))
    elastic = d.user_type == 0
    tx = 0.0
    for m in range(d.M):
        users = r.sel[m]
        mask = users >= 0
        mask[mask] = elastic[users[mask]]
        tx += SITE_ETA[arch][m] * r.slot_power[m][mask].sum()
    assert r.power_sum == pytest.approx(sum(SITE_STATIC[arch]) + tx, rel=1e-12)
    assert r.rate_sum == pytest.approx(r.user_rate[elastic].sum(), rel=1e-12)
    assert r.ee == pytest.approx(r.rate_sum / r.power_sum, rel=1e-12)
    assert tx > 0.0


def test_oma_selects_one_user_per_subcarrier():
    d = synth.architecture_drop("oma", 1, 4)
    r = oracle.solve(d, oracle.Params(fixed_count=0))
    assert r.sel.shape == (d.M, d.N, 1)
    noma = oracle.solve(dataclasses.replace(d, l=2), oracle.Params(fixed_count=0))
    assert ((noma.sel >= 0).sum(axis=2) == 2).any()
