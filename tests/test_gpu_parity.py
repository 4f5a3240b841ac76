"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Every case prints its name before the GPU call so that a failing run names
it.  Inputs come from the seeded generator; expected values from the oracle
(run here, or stored by tests/golden/make_goldens.py for the full-size case).
"""
import hashlib
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import parity, refeval
from tests.drops_util import custom_drop
from tests.gpu_util import gpu_params

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_1803_07772_amd as pa
    assert torch.cuda.is_available()
    c = pa.Context(0)
    yield c
    c.close()


def _run(ctx, d, op, label, device_gain=False, allow_diverged=False, **kw):
    print(f"[gpu case] {label} M={d.M} N={d.N} K={d.K} l={d.l}", flush=True)
    okw = {k: v for k, v in kw.items() if k in ("pmask", "weight", "warm")}
    orc = oracle.solve(d, op, **okw)
    gain = None
    if device_gain:
        import torch
        gain = torch.from_numpy(d.gain).cuda()
    gpu = ctx.solve(d, gpu_params(op), gain=gain, **kw)
    info = parity.compare(d, gpu, orc, pmask=kw.get("pmask"), label=label, allow_diverged=allow_diverged)
    parity.check_structure(d, gpu, kw.get("pmask"))
    print(info, flush=True)
    return gpu, orc, info


def test_cfg1_converge(ctx):
    d = synth.make_drop(synth.CFG1, 0, 0)
    op = oracle.Params(fixed_count=0, sweeps_per_dinkelbach=2000, tol_dinkelbach=1e-6)
    gpu, orc, info = _run(ctx, d, op, "cfg1 seed0 converge")
    assert info["near_ties"] == 0 and gpu.status_flags == 0


def test_cfg2_converge_with_caps(ctx):
    """Seeds 0-15 of the 5-RRH / 64-subcarrier / 32-user configuration: every
    drop at the bars on every element the oracle did not flag; at most one
    drop may take a flagged decision the other way."""
    diverged, flagged = [], 0
    for seed in range(16):
        d = synth.make_drop(synth.CFG2, seed, 0)
        _, _, info = _run(ctx, d, oracle.Params(fixed_count=0), f"cfg2 seed{seed}", device_gain=True,
                          allow_diverged=True)
        flagged += info["flagged_mn"] + info["flagged_users"]
        if info.get("diverged"):
            diverged.append(seed)
    print("cfg2: flagged elements", flagged, "diverged drops", diverged, flush=True)
    assert len(diverged) <= 1


@pytest.mark.parametrize("seed", range(3))
def test_cfg2_fixed_count(ctx, seed):
    d = synth.make_drop(synth.CFG2, 100 + seed, 0)
    _run(ctx, d, oracle.Params(sweeps_per_dinkelbach=100), f"cfg2 fixed seed{100 + seed}")


EDGE = {
    "single_rrh": dict(M=1, N=16, K=8, K_s=2, l=2),
    "oma_l1": dict(M=4, N=24, K=12, K_s=3, l=1),
    "l3_ragged": dict(M=3, N=37, K=37, K_s=9, l=3),
    "l4": dict(M=2, N=9, K=11, K_s=2, l=4),
    "one_subcarrier": dict(M=5, N=1, K=20, K_s=5, l=2),
    "one_user": dict(M=3, N=12, K=1, K_s=0, l=1),
    "all_streaming": dict(M=3, N=16, K=6, K_s=6, l=2),
    "l_equals_K": dict(M=2, N=8, K=3, K_s=1, l=3),
    "wide_K": dict(M=3, N=20, K=1000, K_s=250, l=2),
    "max_M": dict(M=32, N=40, K=100, K_s=25, l=2),
}


@pytest.mark.parametrize("name", sorted(EDGE))
def test_edge_shapes(ctx, name):
    e = EDGE[name]
    rc = synth.CFG2.with_sizes(e["M"], e["N"], e["K"], e["K_s"])
    rc.l = e["l"]
    d = synth.make_drop(rc, 7, 0)
    _run(ctx, d, oracle.Params(sweeps_per_dinkelbach=60, fixed_count=0), f"edge {name}")


def test_weights_and_mask(ctx):
    d = synth.make_drop(synth.CFG2, 11, 0)
    rng = np.random.default_rng(0)
    w = rng.uniform(0.2, 1.0, (d.M, d.K))
    pm = d.pmax_w / d.N * rng.uniform(0.5, 1.5, d.M)
    _run(ctx, d, oracle.Params(sweeps_per_dinkelbach=80), "weights+mask", weight=w, pmask=pm)


def test_warm_start(ctx):
    d = synth.make_drop(synth.CFG2, 12, 0)
    rng = np.random.default_rng(1)
    p0 = np.where(rng.uniform(size=(d.M, d.N, d.K)) < 0.1,
                  rng.uniform(0, 1, (d.M, d.N, d.K)) * (d.pmax_w / d.N)[:, None, None], 0.0)
    warm = dict(p0=p0, xi0=rng.uniform(0, 5, d.M), zeta0=rng.uniform(0, 2, d.K))
    _run(ctx, d, oracle.Params(sweeps_per_dinkelbach=80), "warm start", warm=warm)


def test_sic_pairs_and_refit_period(ctx):
    rng = np.random.default_rng(2)
    M, N, K = 2, 6, 4
    own, near = [0, 0, 1, 1], [1, 0, 1, 0]
    gain = np.empty((M, N, K))
    for m in range(M):
        for k in range(K):
            base = (-10.5 if near[k] else -12.5) if own[k] == m else -13.5
            gain[m, :, k] = 10.0 ** (base + rng.uniform(-0.3, 0.3, N))
    w = np.array([[0.2 if near[k] else 1.0 for k in range(K)] for m in range(M)])
    d = custom_drop(gain, pmax=[6.0, 6.0], eta=[4.0, 2.0], noise=1e-15, l=2)
    _run(ctx, d, oracle.Params(sweeps_per_dinkelbach=150, refit_period=3), "sic pairs", weight=w)


def test_cfg3_full_size_against_stored_oracle(ctx):
    """Full configuration (M=17, N=1024, K=256, l=3, 200 sweeps per step) in the
    launch configuration the benchmark times."""
    g = np.load(os.path.join(GOLD, "cfg3_seed0.npz"))
    d = synth.make_drop(synth.CFG3, 0, 0)
    assert hashlib.sha256(d.gain.tobytes()).digest() == g["gain_sha256"].tobytes()
    import torch

    import paper_1803_07772_amd as pa
    print("[gpu case] cfg3 seed0 full size", flush=True)
    gpu = ctx.solve(d, pa.Params(), gain=torch.from_numpy(d.gain).cuda())

    class O:
        pass
    orc = O()
    orc.sel = g["sel"].astype(np.int32)
    for k in ("slot_power", "rrh_of_user", "xi", "zeta", "zeta_sic", "user_rate", "tie_mn", "tie_user"):
        setattr(orc, k, g[k])
    orc.ee, orc.rate_sum, orc.power_sum, _ = g["scalars"]
    orc.dinkelbach_iters, orc.sweeps, orc.status_flags, orc.near_ties, _ = (int(x) for x in g["ints"])
    info = parity.compare(d, gpu, orc, label="cfg3 seed0")
    parity.check_structure(d, gpu)
    print(info, gpu.status_flags, orc.status_flags, flush=True)
    # the violations of C12-C14 at exit (flags compared by compare() when nothing is flagged)
    vq, vp, vs = g["viol"]
    for x, y in ((gpu.viol_qos, vq), (gpu.viol_budget, vp), (gpu.viol_sic, vs)):
        assert (x == 0) == (y == 0) and abs(x - y) <= 1e-6 * max(abs(y), 1e-300)


def test_deterministic_and_dense_output(ctx):
    d = synth.make_drop(synth.CFG2, 3, 0)
    import paper_1803_07772_amd as pa
    p = pa.Params(sweeps_per_dinkelbach=50)
    print("[gpu case] determinism cfg2 seed3", flush=True)
    a = ctx.solve(d, p, dense_power=True)
    b = ctx.solve(d, p, dense_power=True)
    assert a.ee == b.ee
    assert np.array_equal(a.slot_power, b.slot_power) and np.array_equal(a.sel, b.sel)
    dense = refeval.dense_from_slots(d, a.sel, a.slot_power).astype(np.float32)
    assert np.array_equal(a.power, dense)


def test_invalid_inputs_rejected(ctx):
    import paper_1803_07772_amd as pa
    d = synth.make_drop(synth.CFG1, 0, 0)
    print("[gpu case] invalid inputs", flush=True)
    g = d.gain.copy()
    g[0, 0, 0] = np.nan
    with pytest.raises(pa.AllocError, match="-22"):
        ctx.solve(d, gain=g)
    bad = synth.make_drop(synth.CFG1, 0, 0)
    bad.l = 0
    with pytest.raises(pa.AllocError, match="-22"):
        ctx.solve(bad)
    big = synth.CFG2.with_sizes(33, 4, 8, 2)
    with pytest.raises(pa.AllocError, match="-27"):
        ctx.solve(synth.make_drop(big, 0, 0))
    bad = synth.make_drop(synth.CFG1, 0, 0)
    bad.delay_s = np.zeros_like(bad.delay_s)
    with pytest.raises(pa.AllocError, match="-22"):
        ctx.solve(bad)
    # the context still works after rejected calls
    r = ctx.solve(d, pa.Params(sweeps_per_dinkelbach=5))
    assert np.isfinite(r.ee)
    sys.stdout.flush()


def test_near_tie_reporting(ctx):
    """alloc_params.tie_rel: the GPU counts its own near-tie decisions.  Two
    identical users competing for one subcarrier (l = 1) tie exactly, and
    gains 1e-12 apart are within 1e-9: both are flagged, by the plain and the
    batched solver, as the oracle flags them; gains 1e-3 apart are not.  With
    tie_rel = 0 nothing is counted.  On ordinary drops counting changes no
    result bit, and every drop the GPU flags, the oracle flags too (the GPU
    watches a subset of the oracle's decisions: decoding order and where a
    candidate would enter it, the selection order around the l-th
    candidate, the best two RRHs)."""
    import paper_1803_07772_amd as pa
    from tests.test_oracle_pins import _tie_drop
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=200)
    pt = pa.Params(fixed_count=0, sweeps_per_dinkelbach=200, tie_rel=1e-9)
    for delta, flagged in ((0.0, True), (1e-12, True), (1e-3, False)):
        print(f"[gpu case] near-tie drop delta={delta}", flush=True)
        d = _tie_drop(delta)
        o = oracle.solve(d, oracle.Params(fixed_count=0, sweeps_per_dinkelbach=200), gain=d.gain)
        assert (o.near_ties > 0) == flagged
        for r in (ctx.solve(d, pt), ctx.solve_batch([d], pt)[0]):
            assert (r.near_ties > 0) == flagged, (delta, r.near_ties)
            assert bool(r.status_flags & pa.NEAR_TIE) == flagged
        r0 = ctx.solve(d, p)
        assert r0.near_ties == 0 and not r0.status_flags & pa.NEAR_TIE
    op = oracle.Params(fixed_count=0)
    drops = [synth.make_drop(synth.CFG2, s, 0) for s in range(8)]
    print("[gpu case] near-tie counts on cfg2 seeds 0-7", flush=True)
    a = ctx.solve_batch(drops, gpu_params(op))
    b = ctx.solve_batch(drops, gpu_params(op, tie_rel=1e-9))
    counts = []
    for d, x, y in zip(drops, a, b):
        assert x.ee == y.ee and np.array_equal(x.slot_power, y.slot_power) and x.sweeps == y.sweeps
        assert x.near_ties == 0
        o = oracle.solve(d, op)
        if y.near_ties > 0:
            assert o.near_ties > 0
        counts.append((y.near_ties, o.near_ties))
    print("near ties (gpu, oracle):", counts, flush=True)
