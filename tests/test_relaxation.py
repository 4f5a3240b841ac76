"""The paper's relaxation of the selection constraints against the selection
reading (CPU only).

The method replaces the binary constraints by exact selection: at most l
users per (m,n) and one RRH per user, chosen by the per-triple Lagrangian
maximum.  The paper instead keeps every triple's power and relaxes the
binary constraints into product constraints C10/C11 with their own
multipliers (Sec. II-B, Sec. IV-A); oracle/relaxed.py implements that.  As
rho goes to zero the relaxation's solutions must be allocations that the
selection reading accepts:

* one RRH, NOMA (C11 binds: at most l of three users per subcarrier): the
  relaxation, from an equal share of the mask on every triple, reaches the
  selection method's allocation and EE;
* two RRHs, one user per subcarrier (C10 binds: one RRH per user): the
  relaxation's result meets the product constraints to 10 rho, and the
  selection method started from it (as Dinkelbach's p^0) keeps its users,
  RRHs and EE: each is a fixed point of the selection reading.  Both methods
  are local, and from their cold starts they may settle in different local
  optima; how often they agree is reported, not asserted.
"""
import numpy as np
import pytest

import oracle
from oracle.relaxed import solve_relaxed
from tests import refeval
from tests.drops_util import custom_drop

OP = oracle.Params(fixed_count=0, sweeps_per_dinkelbach=4000, tol_dual=1e-12, tol_dinkelbach=1e-10,
                   max_dinkelbach=40, stall_sweeps=0)
TAU = 1e-2  # a triple carries the user when its power exceeds TAU * mask


def _support(d, P):
    pm = d.pmax_w / d.N
    return P > TAU * pm[:, None, None]


def _one_rrh_noma(seed):
    rng = np.random.default_rng(700 + seed)
    gain = 10.0 ** rng.uniform(-13.5, -11.5, (1, 2, 3))
    return custom_drop(gain, pmax=[2.0], eta=[4.0], noise=1e-15, l=2)


def _two_rrh_ofdma(seed):
    rng = np.random.default_rng(700 + seed)
    gain = 10.0 ** rng.uniform(-13.5, -11.5, (2, 2, 2))
    return custom_drop(gain, pmax=[2.0, 0.5], eta=[4.0, 2.0], noise=1e-15, l=1)


@pytest.mark.parametrize("rho", [1e-4, 1e-6])
def test_relaxation_reaches_the_selection_one_rrh(rho):
    for seed in range(6):
        d = _one_rrh_noma(seed)
        r = oracle.solve(d, OP)
        rx = solve_relaxed(d, rho, rho)
        assert rx["c11_max"] <= 10 * rho
        assert rx["ee"] == pytest.approx(r.ee, rel=1e-5)
        Ps = refeval.dense_from_slots(d, r.sel, r.slot_power)
        assert (_support(d, rx["p"]) == _support(d, Ps)).all(), seed


@pytest.mark.parametrize("rho", [1e-6, 1e-8])
def test_relaxation_results_are_selection_fixed_points_two_rrhs(rho):
    same = 0
    for seed in range(8):
        d = _two_rrh_ofdma(seed)
        rx = solve_relaxed(d, rho, rho)
        assert rx["c10_max"] <= 10 * rho and rx["c11_max"] <= 10 * rho
        rw = oracle.solve(d, OP, warm=dict(p0=rx["p"]))
        Pw = refeval.dense_from_slots(d, rw.sel, rw.slot_power)
        assert (_support(d, Pw) == _support(d, rx["p"])).all(), seed
        assert rw.ee == pytest.approx(rx["ee"], rel=1e-9)
        r = oracle.solve(d, OP)
        same += bool((_support(d, refeval.dense_from_slots(d, r.sel, r.slot_power))
                      == _support(d, rx["p"])).all())
    print(f"rho {rho:g}: cold starts of both methods reach the same decisions on {same} of 8 drops")
