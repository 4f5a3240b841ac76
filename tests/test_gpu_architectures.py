"""GPU parity of the architecture comparison (Sec. VIII): H-CRAN with PD-NOMA,
OMA, 1-tier C-RAN, 2-tier HCN and 1-tier HPN drops of the paper's channel,
through the batched solver (one mixed batch) and the plain solver, each drop
against the FP64 oracle."""
import dataclasses

import pytest

import oracle
import synth
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_1803_07772_amd as pa
    assert torch.cuda.is_available()
    c = pa.Context(0)
    yield c
    c.close()


def _check(drops, results, op):
    """Every drop at the bars of tests/parity.py on every element the oracle
    did not flag; returns (drops with flagged elements, drops where a flagged
    decision went the other way)."""
    flagged = diverged = 0
    for d, r in zip(drops, results):
        o = oracle.solve(d, op)
        info = parity.compare(d, r, o, label=f"{d.M}x{d.N}x{d.K} l={d.l} index {d.index}",
                              allow_diverged=True)
        parity.check_structure(d, r)
        print(info, flush=True)
        flagged += info["flagged_mn"] + info["flagged_users"] > 0
        diverged += bool(info.get("diverged"))
    return flagged, diverged


def test_architectures_batched(ctx):
    import torch

    import paper_1803_07772_amd as pa
    drops = [synth.architecture_drop(a, 5, i) for a in synth.ARCHITECTURES for i in range(6)]
    print(f"[gpu case] architecture batch of {len(drops)} drops", flush=True)
    gains = [torch.from_numpy(d.gain).cuda() for d in drops]
    res = ctx.solve_batch(drops, pa.Params(fixed_count=0), gains=gains)
    flagged, diverged = _check(drops, res, oracle.Params(fixed_count=0))
    print("architecture batch: drops with flagged elements", flagged, "diverged", diverged, flush=True)
    assert diverged <= 1


@pytest.mark.parametrize("arch", synth.ARCHITECTURES)
def test_architectures_plain(ctx, arch):
    import paper_1803_07772_amd as pa
    d = synth.architecture_drop(arch, 5, 0)
    print(f"[gpu case] plain {arch}", flush=True)
    r = ctx.solve(d, pa.Params(fixed_count=0))
    flagged, diverged = _check([d], [r], oracle.Params(fixed_count=0))
    assert diverged == 0


def test_trend_study_points(ctx):
    """Corner points of the trend studies run by bench.py --sweeps: most users
    and LPNs, the highest arrival rate, OMA."""
    import paper_1803_07772_amd as pa
    base = synth.PAPER
    rcs = [dataclasses.replace(base, K=28, K_s=2), dataclasses.replace(base, K=28, K_s=6,
                                                                       rate_bps_lo=256e3, rate_bps_hi=256e3),
           dataclasses.replace(base, M=7, K=12, K_s=6), dataclasses.replace(base, M=7, K=12, K_s=6, l=1),
           dataclasses.replace(base, K=28, K_s=6, l=1)]
    drops = [synth.make_drop(rc, 0, i) for rc in rcs for i in range(4)]
    print(f"[gpu case] trend-study batch of {len(drops)} drops", flush=True)
    res = ctx.solve_batch(drops, pa.Params(fixed_count=0))
    flagged, diverged = _check(drops, res, oracle.Params(fixed_count=0))
    print("trend points: drops with flagged elements", flagged, "diverged", diverged, flush=True)
    assert diverged <= 1
