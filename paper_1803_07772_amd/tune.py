"""Autotuner of the batched solver's launch shape.

The choices are the LDS share of a workgroup (``lds_kb``: a whole compute
unit, or a half, a third or a quarter so that several workgroups share one),
the cap on subcarriers per LDS tile (``tile``) and the threads per workgroup
(``block``: 512, 256 for more and smaller workgroups per compute unit, or
1024 for one workgroup per compute unit with all of its LDS) and
whether each wave runs its own subcarriers (``wave``: subcarriers per wave
tile, 0 = tiles of the whole workgroup).  They change only the order of
floating-point sums inside a drop, not the method.  Candidates are timed on
the GPU (the batched kernel's HIP-event duration) on the whole batch, so the
load per workgroup (and which drops are split over several workgroups) is the
real one, but with a short fixed schedule (a few sweeps, every drop the same
count) to keep tuning cheap; the fastest per size bucket is kept in a JSON
cache that later batches of the same bucket reuse.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os

import numpy as np

from . import Params

CANDIDATES = (
    {"lds_kb": 0, "tile": 0, "block": 512, "wave": 0},
    {"lds_kb": 79, "tile": 0, "block": 512, "wave": 0},
    {"lds_kb": 52, "tile": 0, "block": 512, "wave": 0},
    {"lds_kb": 0, "tile": 8, "block": 512, "wave": 0},
    {"lds_kb": 79, "tile": 8, "block": 512, "wave": 0},
    {"lds_kb": 79, "tile": 0, "block": 256, "wave": 0},
    {"lds_kb": 52, "tile": 0, "block": 256, "wave": 0},
    {"lds_kb": 39, "tile": 0, "block": 256, "wave": 0},
    {"lds_kb": 0, "tile": 8, "block": 256, "wave": 0},
    {"lds_kb": 0, "tile": 0, "block": 512, "wave": 1},
    {"lds_kb": 0, "tile": 0, "block": 256, "wave": 1},
    {"lds_kb": 0, "tile": 0, "block": 512, "wave": 2},
    {"lds_kb": 0, "tile": 0, "block": 256, "wave": 2},
    {"lds_kb": 0, "tile": 0, "block": 1024, "wave": 0},
    {"lds_kb": 0, "tile": 8, "block": 1024, "wave": 0},
)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def _up2(x: int) -> int:
    return 1 << max(0, math.ceil(math.log2(max(1, x))))


def bucket(M: int, N: int, K: int, l: int) -> str:
    """Size class: M, N and K rounded up to powers of two, and l."""
    return f"M{_up2(M)}-N{_up2(N)}-K{_up2(K)}-l{l}"


def batch_key(drops) -> str:
    """Bucket of the drop at the middle of the batch's work (M N K)."""
    w = np.array([d.M * d.N * d.K for d in drops], float)
    order = np.argsort(w, kind="stable")
    c = np.cumsum(w[order])
    mid = drops[int(order[np.searchsorted(c, 0.5 * c[-1])])]
    return bucket(mid.M, mid.N, mid.K, mid.l)


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_cache(cache: dict, path: str = DEFAULT_CACHE):
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
        f.write("\n")


def tuned(drops, params: Params, cache: dict | None = None) -> Params:
    """params with the cached launch shape of the batch's bucket (unchanged
    when the bucket was never tuned)."""
    cache = load_cache() if cache is None else cache
    e = cache.get(batch_key(drops))
    if not e:
        return params
    return dataclasses.replace(params, lds_kb=int(e["lds_kb"]), tile=int(e["tile"]),
                               block=int(e.get("block", 0)), wave=int(e.get("wave", 0)))


def tune(ctx, drops, params: Params, gains=None, sweeps: int = 12,
         candidates=CANDIDATES, cache: dict | None = None):
    """Times every candidate on the batch with a fixed schedule of ``sweeps``
    sweeps in each of two Dinkelbach steps; returns (best, timings) and
    records the best under the batch's bucket in ``cache`` if given."""
    short = dataclasses.replace(params, fixed_count=1, sweeps_per_dinkelbach=sweeps, max_dinkelbach=2)
    was = ctx.timing
    ctx.set_timing(True)
    times = []
    for cand in candidates:
        p = dataclasses.replace(short, **cand)
        ctx.solve_batch(drops, dataclasses.replace(p, sweeps_per_dinkelbach=1, max_dinkelbach=1), gains=gains)
        ctx.solve_batch(drops, p, gains=gains)
        times.append((ctx.last_kernel_ms(), cand))
    ctx.set_timing(was)
    # candidates are in order of preference: keep the first within 2% of the
    # fastest (the short schedule cannot separate closer ones)
    fastest = min(t for t, _ in times)
    best = next(c for t, c in times if t <= 1.02 * fastest)
    if cache is not None:
        cache[batch_key(drops)] = dict(best, ms={"/".join(str(c[f]) for f in ("lds_kb", "tile", "block", "wave")): round(t, 3)
                                                 for t, c in times},
                                      drops=len(drops), sweeps=sweeps)
    return best, times
