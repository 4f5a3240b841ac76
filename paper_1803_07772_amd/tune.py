"""Autotuner of the batched solver's launch shape.

The choices are the LDS share of a workgroup (``lds_kb``: a whole compute
unit, or a half, a third or a quarter so that several workgroups share one),
the cap on subcarriers per LDS tile (``tile``) and the threads per workgroup
(``block``: 512, 256 for more and smaller workgroups per compute unit, or
1024 for one workgroup per compute unit with all of its LDS) and
whether each wave runs its own subcarriers (``wave``: subcarriers per wave
tile, 0 = tiles of the whole workgroup), and the schedule: how many
workgroups solve a large drop together (``group_triples``: a drop of more
triples is split over about triples/group_triples workgroups; 0 = the
library's rule by the average load).  They change only the order of
floating-point sums inside a drop, not the method.

Candidates are timed on the GPU (the batched kernel's HIP-event duration) on
the whole batch, so the load per workgroup is the real one.  The launch
shapes are first timed with a short fixed schedule (a few sweeps, every drop
the same count), which ranks the per-sweep cost; the leading shapes are then
timed with the real schedule, each with every group_triples candidate,
because the end of a launch is set by the drops that need the most sweeps,
which only full solves show.  The fastest per size bucket is kept in a JSON
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
                               block=int(e.get("block", 0)), wave=int(e.get("wave", 0)),
                               group_triples=int(e.get("group_triples", 0)))


SHAPE_FIELDS = ("lds_kb", "tile", "block", "wave")


def group_candidates(drops) -> list:
    """Schedules to try: the library's rule (0), and splitting every drop
    above a half, a quarter and an eighth of the largest drop's triples."""
    big = max(d.M * d.N * d.K for d in drops)
    return [0] + sorted({max(1, big // f) for f in (2, 4, 8)}, reverse=True)


def tune(ctx, drops, params: Params, gains=None, sweeps: int = 12,
         candidates=CANDIDATES, cache: dict | None = None, full: int = 3, groups=None):
    """Times every launch shape on the batch with a fixed schedule of
    ``sweeps`` sweeps in each of two Dinkelbach steps, then the ``full``
    fastest of them with the real schedule ``params`` under every schedule of
    ``groups`` (default group_candidates(drops)); ``full`` = 0 keeps the
    short ranking alone.  Returns (best, timings) and records the best under
    the batch's bucket in ``cache`` if given."""
    short = dataclasses.replace(params, fixed_count=1, sweeps_per_dinkelbach=sweeps, max_dinkelbach=2)
    was = ctx.timing
    ctx.set_timing(True)
    times = []
    for cand in candidates:
        p = dataclasses.replace(short, **cand)
        ctx.solve_batch(drops, dataclasses.replace(p, sweeps_per_dinkelbach=1, max_dinkelbach=1), gains=gains)
        ctx.solve_batch(drops, p, gains=gains)
        times.append((ctx.last_kernel_ms(), cand))
    # candidates are in order of preference: keep the first within 2% of the
    # fastest (the short schedule cannot separate closer ones)
    fastest = min(t for t, _ in times)
    best = dict(next(c for t, c in times if t <= 1.02 * fastest), group_triples=0)
    full_times = []
    if full > 0:
        lead = [c for _, c in sorted(times, key=lambda x: x[0])[:full]]
        for cand in lead:
            for g in (group_candidates(drops) if groups is None else groups):
                p = dataclasses.replace(params, **cand, group_triples=g)
                ctx.solve_batch(drops, p, gains=gains)
                full_times.append((ctx.last_kernel_ms(), dict(cand, group_triples=g)))
        best = min(full_times, key=lambda x: x[0])[1]
    ctx.set_timing(was)
    if cache is not None:
        key = lambda c: "/".join(str(c[f]) for f in SHAPE_FIELDS)  # noqa: E731
        cache[batch_key(drops)] = dict(
            best, ms={key(c): round(t, 3) for t, c in times},
            full_ms={key(c) + f"/g{c['group_triples']}": round(t, 3) for t, c in full_times},
            drops=len(drops), sweeps=sweeps)
    return best, times + full_times
