"""The global solver (monotonic optimization, Sec. IV-B) and the optimality gap
of the suboptimal method (CPU only).

The global solver (oracle/polyblock.py) is pinned to what the mathematics
fixes: the Lambert-W optimum of a single link, the EE water-filling optimum
of one RRH with one user per subcarrier, brute force over gridded powers on
2 x 2 x 2 drops (any grid point it finds feasible is a lower bound of the
optimum) and the independent evaluator's EE and feasibility of the
allocation it returns.  Both of its algorithms (the polyblock and
branch-reduce-and-bound) are pinned to the closed forms; the polyblock only
where its canonical form has at most three dimensions, since its outer
approximation converges too slowly beyond.  Then the suboptimal method's EE
is compared with the certified optimum.
"""
import numpy as np
import pytest

import oracle
from oracle import polyblock as pb
from tests import refeval
from tests.drops_util import custom_drop, psi_of
from tests.test_oracle_pins import _brute_force, _lambert_opt, _water_filling

EPS = 1e-3  # relative tolerance of the parametric problems


def _check_solution(d, r, psi=None):
    """The returned allocation is feasible and its EE, by the independent
    evaluator, is the solver's lower end."""
    P = r["power"]
    ok = refeval.feasibility(d, P, d.l, psi=psi, qos_rel=1e-9, tol=1e-9)
    assert all(ok.values()), ok
    assert refeval.evaluate(d, P)["ee"] == pytest.approx(r["ee_lo"], rel=1e-9)


@pytest.mark.parametrize("method", ["polyblock", "brb"])
@pytest.mark.parametrize("pmax", [39.8, 0.05])
def test_single_link_lambert_w(method, pmax):
    """M=N=K=1: the certified interval holds the Lambert-W optimum, and the
    allocation found reaches it (interior optimum, and the mask-bound one)."""
    sg, g = 1e-15, 1e-12
    d = custom_drop(np.full((1, 1, 1), g), pmax=[pmax], eta=[4.0], noise=sg, l=1)
    _, e_star = _lambert_opt(float(np.float32(g)) / sg, refeval.static_power(d), 4.0, pmax)
    r = pb.global_optimum(d, rel_eps=EPS, method=method)
    assert r["ee_lo"] <= e_star * (1 + 1e-12) <= r["ee_hi"] * (1 + 1e-12)
    assert r["ee_lo"] == pytest.approx(e_star, rel=1e-6)
    assert r["ee_hi"] <= e_star * (1 + 3 * EPS)
    _check_solution(d, r)


@pytest.mark.parametrize("method,N,K", [("polyblock", 1, 2), ("brb", 2, 2), ("brb", 3, 2)])
def test_one_rrh_water_filling(method, N, K):
    """M=1, l=1, elastic users: the optimum gives each subcarrier to its best
    user at the water-filling power of the optimal E (a textbook closed form
    with E found by bisection).  The polyblock runs where its canonical form
    has at most three dimensions (it converges slowly beyond)."""
    rng = np.random.default_rng(100)
    gain = 10.0 ** rng.uniform(-13.5, -12.0, (1, N, K))
    d = custom_drop(gain, pmax=[2.0], eta=[4.0], noise=1e-15, l=1)
    best, p_wf, E_wf = _water_filling(d)
    r = pb.global_optimum(d, rel_eps=EPS, method=method)
    assert r["ee_lo"] <= E_wf * (1 + 1e-9) and E_wf <= r["ee_hi"] * (1 + 1e-12)
    assert r["ee_lo"] == pytest.approx(E_wf, rel=1e-6)
    assert r["ee_hi"] <= E_wf * (1 + 3 * EPS)
    _check_solution(d, r)
    for n in range(N):
        if p_wf[n] > 0:
            assert r["power"][0, n, best[n]] == pytest.approx(p_wf[n], rel=1e-2)


def _tiny(seed, M=2, N=2, K=2):
    rng = np.random.default_rng(500 + seed)
    gain = 10.0 ** rng.uniform(-13.5, -11.5, (M, N, K))
    ut = [0] * (K - 1) + [1] if seed % 2 else [0] * K
    return custom_drop(gain, user_type=ut, pmax=[2.0, 0.5, 1.0][:M], eta=[4.0, 2.0, 2.0][:M],
                       noise=1e-15, l=2, arrival=[0.0] * (K - 1) + [64e3], delay=[0.0] * (K - 1) + [0.1])


TINY_EPS = 3e-3
TINY_BOXES = 30000  # per pattern and parametric problem


@pytest.mark.slow
@pytest.mark.parametrize("seed", [0, 1, 3])
def test_global_optimum_bounds_brute_force(seed):
    """2 x 2 x 2 drops (l = 2, a streaming user in odd seeds): the best
    gridded allocation (9 levels per power, refined) is a feasible point, so
    it lies below the certified upper end.  Where the solve completes (the
    streaming drops here) its allocation is at least as good, up to the
    grid's resolution."""
    d = _tiny(seed)
    psi = psi_of(d)
    r = pb.global_optimum(d, rel_eps=TINY_EPS, method="brb", max_iter=TINY_BOXES)
    e_bf, _ = _brute_force(d, psi, levels=9)
    print("seed", seed, "brute force", e_bf, "certified", r["ee_lo"], r["ee_hi"])
    assert e_bf <= r["ee_hi"] * (1 + 1e-9)
    if seed % 2:
        assert r["ee_hi"] <= r["ee_lo"] * (1 + 3 * TINY_EPS)
        assert r["ee_lo"] >= e_bf * (1 - 1e-3)
    _check_solution(d, r, psi)


@pytest.mark.slow
def test_optimality_gap_of_the_method():
    """The suboptimal method (the oracle's Dinkelbach-SCALE-dual solve) on
    2 x 2 x 2 drops against the certified optimum: never above it, and the
    gap is reported as an interval (the optimum lies between the best
    allocation found and the certified upper end).  The method is local, so
    the bar on the ratios is soft."""
    lo, hi = [], []
    for seed in range(8):
        d = _tiny(seed)
        ro = oracle.solve(d, oracle.Params(fixed_count=0))
        P = refeval.dense_from_slots(d, ro.sel, ro.slot_power)
        r = pb.global_optimum(d, rel_eps=TINY_EPS, start=P, method="brb", max_iter=TINY_BOXES)
        assert r["feasible"]
        assert ro.ee <= r["ee_hi"] * (1 + 1e-9)
        assert r["ee_lo"] >= ro.ee * (1 - 1e-12)
        _check_solution(d, r, psi_of(d))
        lo.append(ro.ee / r["ee_hi"])
        hi.append(ro.ee / r["ee_lo"])
    lo, hi = np.array(lo), np.array(hi)
    print("EE of the method / optimum, between", np.round(lo, 3), "and", np.round(hi, 3))
    assert np.median(lo) >= 0.7
