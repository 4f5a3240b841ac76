"""GPU parity of the batched persistent solver (through alloc_solve_batch)."""
import dataclasses
import os

import numpy as np
import pytest

import oracle
import synth
from tests import parity
from tests.gpu_util import gpu_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_1803_07772_amd as pa
    assert torch.cuda.is_available()
    c = pa.Context(0)
    yield c
    c.close()


def _mixed_batch():
    """Ragged sizes: small, medium, one subcarrier, one user, l = 1..4."""
    shapes = [(3, 8, 6, 2, 2), (5, 64, 32, 8, 2), (2, 1, 7, 2, 2), (4, 12, 1, 0, 1),
              (3, 37, 37, 9, 3), (2, 9, 11, 2, 4), (1, 16, 8, 2, 2), (6, 128, 48, 12, 3),
              (5, 64, 32, 8, 2), (4, 24, 12, 3, 1), (8, 33, 70, 17, 3), (3, 5, 9, 9, 2)]
    drops = []
    for i, (M, N, K, Ks, l) in enumerate(shapes):
        rc = synth.CFG2.with_sizes(M, N, K, Ks)
        rc.l = l
        drops.append(synth.make_drop(rc, 40 + i, i))
    return drops


def test_batch_matches_oracle_per_drop(ctx):
    import torch

    import paper_1803_07772_amd as pa
    drops = _mixed_batch()
    op = oracle.Params(fixed_count=0, sweeps_per_dinkelbach=120)
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=120)
    print(f"[gpu case] batch of {len(drops)} mixed drops", flush=True)
    gains = [torch.from_numpy(d.gain).cuda() for d in drops]
    res = ctx.solve_batch(drops, p, gains=gains)
    diverged = 0
    for d, r in zip(drops, res):
        o = oracle.solve(d, op)
        info = parity.compare(d, r, o, label=f"batch drop {d.index} {d.M}x{d.N}x{d.K} l={d.l}",
                              allow_diverged=True)
        parity.check_structure(d, r)
        print(info, flush=True)
        diverged += bool(info.get("diverged"))
    assert diverged <= 1


def test_batch_host_gains_and_dense(ctx):
    import paper_1803_07772_amd as pa
    drops = _mixed_batch()[:4]
    print("[gpu case] batch host gains", flush=True)
    res = ctx.solve_batch(drops, pa.Params(sweeps_per_dinkelbach=30), dense_power=True)
    for d, r in zip(drops, res):
        dense = np.zeros((d.M, d.N, d.K), np.float32)
        for m in range(d.M):
            for n in range(d.N):
                for a in range(d.l):
                    if r.sel[m, n, a] >= 0:
                        dense[m, n, r.sel[m, n, a]] = r.slot_power[m, n, a]
        assert np.array_equal(dense, r.power)


def test_batch_agrees_with_plain_solver(ctx):
    """Same method, same schedule: the batched and the grid solver agree."""
    import paper_1803_07772_amd as pa
    drops = [synth.make_drop(synth.CFG2, s, 0) for s in (0, 1, 2, 4)]
    p = pa.Params(sweeps_per_dinkelbach=100)
    print("[gpu case] batch vs plain", flush=True)
    res = ctx.solve_batch(drops, p)
    for d, rb in zip(drops, res):
        rp = ctx.solve(d, p)
        assert rb.ee == pytest.approx(rp.ee, rel=1e-9)
        assert np.array_equal(rb.sel, rp.sel)
        assert np.array_equal(rb.rrh_of_user, rp.rrh_of_user)
        np.testing.assert_allclose(rb.slot_power, rp.slot_power, rtol=1e-7, atol=1e-15)


def test_batch_cfg4_generator_subset(ctx):
    """Drops of the ragged 4096-drop configuration's generator, the smallest
    and the largest of 64 among them, solved in one batch: every drop
    against the oracle."""
    import torch

    import paper_1803_07772_amd as pa
    M, N, K = synth.batch_sizes(64, seed=0)
    work = M * N * K
    idx = sorted(set([b for b in range(64) if work[b] <= 60000][:5] + [int(np.argmax(work))]))
    drops = synth.make_batch(64, seed=0, indices=idx)
    print(f"[gpu case] cfg4 subset sizes {[(d.M, d.N, d.K) for d in drops]}", flush=True)
    gains = [torch.from_numpy(d.gain).cuda() for d in drops]
    op = oracle.Params(fixed_count=0, sweeps_per_dinkelbach=60)
    res = ctx.solve_batch(drops, gpu_params(op), gains=gains)
    diverged = 0
    for d, r in zip(drops, res):
        o = oracle.solve(d, op)
        info = parity.compare(d, r, o, label=f"cfg4 drop {d.index} {d.M}x{d.N}x{d.K}", allow_diverged=True)
        parity.check_structure(d, r)
        print(info, flush=True)
        diverged += bool(info.get("diverged"))
    assert diverged <= 1


def test_batch_rejects_bad_drop(ctx):
    import paper_1803_07772_amd as pa
    drops = _mixed_batch()[:3]
    bad = dataclasses.replace(drops[1], l=0)
    print("[gpu case] batch invalid", flush=True)
    with pytest.raises(pa.AllocError, match="-22"):
        ctx.solve_batch([drops[0], bad, drops[2]])


def test_batch_warm_starts_match_oracle(ctx):
    """Warm starts (initial powers and multipliers, or multipliers only) in a
    batch, against the oracle from the same warm start; cold drops in between."""
    import paper_1803_07772_amd as pa
    drops = _mixed_batch()[:8]
    rng = np.random.default_rng(5)
    warms = []
    for i, d in enumerate(drops):
        if i % 3 == 2:
            warms.append(None)
            continue
        w = dict(xi0=rng.uniform(0, 3, d.M), zeta0=rng.uniform(0, 2, d.K))
        if i % 3 == 0:
            pm = d.pmax_w / d.N
            w["p0"] = np.where(rng.uniform(size=(d.M, d.N, d.K)) < 0.2,
                               rng.uniform(0, 1.2, (d.M, d.N, d.K)) * pm[:, None, None], 0.0)
        warms.append(w)
    op = oracle.Params(fixed_count=0, sweeps_per_dinkelbach=80)
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=80)
    print(f"[gpu case] batch of {len(drops)} drops with warm starts", flush=True)
    res = ctx.solve_batch(drops, p, warms=warms)
    diverged = 0
    for d, w, r in zip(drops, warms, res):
        o = oracle.solve(d, op, warm=w)
        info = parity.compare(d, r, o, label=f"warm batch drop {d.index} warm={sorted(w or {})}",
                              allow_diverged=True)
        print(info, flush=True)
        diverged += bool(info.get("diverged"))
    assert diverged <= 1


def _same(a, b):
    for k in ("sel", "slot_power", "rrh_of_user", "xi", "zeta"):
        u, v = getattr(a, k), getattr(b, k)
        bad = np.argwhere(u != v)
        if len(bad):
            i = tuple(bad[0])
            print(f"{k}: {len(bad)} entries differ, first {i}: {u[i]!r} vs {v[i]!r}", flush=True)
    assert a.ee == b.ee and a.status_flags == b.status_flags
    assert a.sweeps == b.sweeps and a.dinkelbach_iters == b.dinkelbach_iters
    assert np.array_equal(a.sel, b.sel) and np.array_equal(a.slot_power, b.slot_power)
    assert np.array_equal(a.rrh_of_user, b.rrh_of_user) and np.array_equal(a.xi, b.xi)


def test_graph_batch_replays_match_eager(ctx):
    """The captured batch (alloc_batch_*) replayed three times, with eager
    solves in between: every replay equals the eager batched solve."""
    import torch

    import paper_1803_07772_amd as pa
    drops = _mixed_batch()
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=60)
    gains = [torch.from_numpy(d.gain).cuda() for d in drops]
    print(f"[gpu case] graph batch of {len(drops)} drops, 3 replays", flush=True)
    eager = ctx.solve_batch(drops, p, gains=gains)
    bt = pa.Batch(ctx, drops, p, gains=gains)
    for rep in range(3):
        bt.run()
        got = bt.results()
        for a, b in zip(got, eager):
            _same(a, b)
        ctx.solve(drops[rep], p)  # eager work between replays
        torch.cuda.synchronize()
    bt.close()
    # host gains are copied in at creation (compared with the same four-drop
    # batch: how many workgroups share a drop depends on the batch)
    bh = pa.Batch(ctx, drops[:4], p)
    bh.run()
    for a, b in zip(bh.results(), ctx.solve_batch(drops[:4], p)):
        _same(a, b)
    bh.close()


def test_lds_cap_shares_compute_units(ctx):
    """A smaller LDS share per workgroup (smaller tiles, two workgroups per
    compute unit) gives the same allocations up to the order of the tile sums."""
    import paper_1803_07772_amd as pa
    drops = [synth.make_drop(synth.CFG2, 60 + i, i) for i in range(6)]
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=60)
    print("[gpu case] batch with lds_kb=64", flush=True)
    full = ctx.solve_batch(drops, p)
    capped = ctx.solve_batch(drops, dataclasses.replace(p, lds_kb=64))
    for a, b in zip(capped, full):
        assert abs(a.ee - b.ee) <= 1e-9 * abs(b.ee)
        assert np.array_equal(a.sel, b.sel) and np.array_equal(a.rrh_of_user, b.rrh_of_user)
    # 256-thread workgroups (more, smaller workgroups per compute unit) and
    # 1024-thread ones (one per compute unit, all of its LDS)
    for blk, kb in ((256, 39), (1024, 0)):
        for a, b in zip(ctx.solve_batch(drops, dataclasses.replace(p, block=blk, lds_kb=kb)), full):
            assert abs(a.ee - b.ee) <= 1e-9 * abs(b.ee)
            assert np.array_equal(a.sel, b.sel) and np.array_equal(a.rrh_of_user, b.rrh_of_user)
    with pytest.raises(pa.AllocError, match="-22"):
        ctx.solve_batch(drops[:1], dataclasses.replace(p, block=128))
    # a share below what a drop needs is raised to that need
    tiny = ctx.solve_batch(drops[:2], dataclasses.replace(p, lds_kb=2))
    for a, b in zip(tiny, full[:2]):
        assert abs(a.ee - b.ee) <= 1e-9 * abs(b.ee)
        assert np.array_equal(a.sel, b.sel)


def test_wave_tiles_match_oracle(ctx):
    """Each wave running its own subcarriers (no workgroup barrier inside a
    pass) on ragged drops, including drops with fewer subcarriers than waves:
    parity with the oracle per drop."""
    import torch

    import paper_1803_07772_amd as pa
    drops = _mixed_batch()
    op = oracle.Params(fixed_count=0, sweeps_per_dinkelbach=120)
    # three workgroups in all: no drop is split over several
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=120, max_groups=3)
    gains = [torch.from_numpy(d.gain).cuda() for d in drops]
    orcs = [oracle.solve(d, op) for d in drops]
    for wave, blk in ((1, 0), (2, 256)):
        print(f"[gpu case] wave tiles: wave={wave} block={blk}, {len(drops)} mixed drops", flush=True)
        res = ctx.solve_batch(drops, dataclasses.replace(p, wave=wave, block=blk), gains=gains)
        diverged = 0
        for d, r, o in zip(drops, res, orcs):
            info = parity.compare(d, r, o, label=f"wave={wave} drop {d.index} {d.M}x{d.N}x{d.K} l={d.l}",
                                  allow_diverged=True)
            print(info, flush=True)
            diverged += bool(info.get("diverged"))
        assert diverged <= 1


def test_wave_tiles_agree_with_workgroup_tiles(ctx):
    """Wave tiles only change the order of the sums over subcarriers: the
    same allocations as workgroup tiles; replays of a captured wave-tiled
    batch equal the eager solve."""
    import paper_1803_07772_amd as pa
    drops = [synth.make_drop(synth.CFG2, 70 + i, i) for i in range(6)]
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=60, max_groups=6)
    print("[gpu case] wave tiles vs workgroup tiles, 6 drops", flush=True)
    ref = ctx.solve_batch(drops, p)
    for wave, blk in ((1, 0), (2, 0), (1, 256), (4, 256)):
        q = dataclasses.replace(p, wave=wave, block=blk)
        for a, b in zip(ctx.solve_batch(drops, q), ref):
            assert abs(a.ee - b.ee) <= 1e-9 * abs(b.ee), (wave, blk)
            assert np.array_equal(a.sel, b.sel) and np.array_equal(a.rrh_of_user, b.rrh_of_user)
    with pytest.raises(pa.AllocError, match="-22"):
        ctx.solve_batch(drops[:1], dataclasses.replace(p, wave=17))
    q = dataclasses.replace(p, wave=1)
    eager = ctx.solve_batch(drops, q)
    bt = pa.Batch(ctx, drops, q)
    for rep in range(2):
        bt.run()
        for a, b in zip(bt.results(), eager):
            _same(a, b)
    bt.close()


def test_autotuner_picks_a_candidate(ctx):
    import paper_1803_07772_amd as pa
    from paper_1803_07772_amd import tune
    drops = [synth.make_drop(synth.CFG2, 80 + i, i) for i in range(24)]
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=40)
    print("[gpu case] autotuner on 24 drops", flush=True)
    cache = {}
    best, times = tune.tune(ctx, drops, p, sweeps=4, cache=cache, full=2)
    shape = {f: best[f] for f in tune.SHAPE_FIELDS}
    assert shape in tune.CANDIDATES and best["group_triples"] in tune.group_candidates(drops)
    assert len(times) == len(tune.CANDIDATES) + 2 * len(tune.group_candidates(drops))
    assert all(t > 0 for t, _ in times)
    key = tune.batch_key(drops)
    assert all(cache[key][f] == best[f] for f in ("lds_kb", "tile", "block", "wave", "group_triples"))
    q = tune.tuned(drops, p, cache)
    ref = ctx.solve_batch(drops[:4], p)
    for a, b in zip(ctx.solve_batch(drops[:4], q), ref):
        assert abs(a.ee - b.ee) <= 1e-9 * abs(b.ee)


def test_group_scheduled_large_drop_matches_oracle(ctx):
    """A drop far above the average load is split over many workgroups that
    meet at a group barrier; small drops around it stay one per workgroup."""
    import torch

    import paper_1803_07772_amd as pa
    rc = synth.CFG2.with_sizes(6, 256, 64, 16)
    rc.l = 3
    big = synth.make_drop(rc, 5, 0)
    small = [synth.make_drop(synth.CFG1, s, 0) for s in range(5)]
    drops = [small[0], big] + small[1:]
    op = oracle.Params(fixed_count=0, sweeps_per_dinkelbach=60)
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=60)
    print("[gpu case] group-scheduled drop 6x256x64 l=3 among 5 small drops", flush=True)
    res = ctx.solve_batch(drops, p, gains=[torch.from_numpy(d.gain).cuda() for d in drops])
    for d, r in zip(drops, res):
        o = oracle.solve(d, op)
        info = parity.compare(d, r, o, label=f"group batch {d.M}x{d.N}x{d.K}")
        parity.check_structure(d, r)
        print(info, flush=True)
    # the same drop alone (one drop: as many ranks as fit), with a small cap on
    # the grid, and through the plain solver: the same allocation
    alone = ctx.solve_batch([big], p)[0]
    capped = ctx.solve_batch(drops, dataclasses.replace(p, max_groups=3))[1]
    plain = ctx.solve(big, p)
    # 1024-thread workgroups with a whole compute unit's LDS each
    wide = ctx.solve_batch(drops, dataclasses.replace(p, block=1024))[1]
    for x in (alone, capped, plain, wide):
        assert abs(x.ee - res[1].ee) <= 1e-9 * abs(res[1].ee)
        assert np.array_equal(x.sel, res[1].sel) and np.array_equal(x.rrh_of_user, res[1].rrh_of_user)


def test_association_sums_in_device_memory(ctx):
    """A 17 x 64 x 256 drop fits one subcarrier per 1024-thread workgroup's
    tile with its M*K association sums in LDS and two with them in device
    memory, which the solvers then choose.  Solved by one workgroup and by
    four (batched solver) and by sixteen (grid solver), with the sums in
    device memory and, under a tile cap of one, in LDS: every case against
    the oracle."""
    import torch

    import paper_1803_07772_amd as pa
    rc = synth.CFG3.with_sizes(17, 64, 256, 64)
    rc.l = 3
    d = synth.make_drop(rc, 7, 0)
    o = oracle.solve(d, oracle.Params(fixed_count=0, sweeps_per_dinkelbach=60))
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=60, block=1024)
    g = torch.from_numpy(d.gain).cuda()
    for where, tile in (("device memory", 0), ("LDS", 1)):
        for groups in (1, 4, 16):
            q = dataclasses.replace(p, max_groups=groups, tile=tile)
            print(f"[gpu case] 17x64x256 l=3, sums in {where}, {groups} workgroups", flush=True)
            if groups == 16:
                r = ctx.solve(d, q, gain=g)
            else:
                r = ctx.solve_batch([d], q, gains=[g])[0]
            info = parity.compare(d, r, o, label=f"sums in {where}, {groups} workgroups")
            parity.check_structure(d, r)
            print(info, flush=True)


def test_group_scheduled_graph_replays(ctx):
    """Group barriers start each replay from zero arrivals."""
    import paper_1803_07772_amd as pa
    rc = synth.CFG2.with_sizes(5, 128, 32, 8)
    drops = [synth.make_drop(rc, 9, 0)] + [synth.make_drop(synth.CFG1, s, 0) for s in range(3)]
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=40)
    print("[gpu case] group-scheduled graph replays", flush=True)
    eager = ctx.solve_batch(drops, p)
    bt = pa.Batch(ctx, drops, p)
    for _ in range(3):
        bt.run()
        for a, b in zip(bt.results(), eager):
            _same(a, b)
    bt.close()


def test_benchmark_batch_full_size(ctx):
    """The benchmark's workload at full size and in its launch shape: 4096
    drops of 5 RRHs x 64 subcarriers x 32 users, one graph replay in the
    tuned shape.  A seeded sample of 16 drops against the oracle; every drop
    against the properties any allocation has."""
    import torch

    import paper_1803_07772_amd as pa
    from paper_1803_07772_amd import tune
    drops = [synth.make_drop(synth.CFG2, s, 0) for s in range(4096)]
    gains = [torch.from_numpy(d.gain).cuda() for d in drops]
    p = tune.tuned(drops, pa.Params(fixed_count=0))
    print(f"[gpu case] 4096-drop batch, lds_kb={p.lds_kb} block={p.block} wave={p.wave}", flush=True)
    bt = pa.Batch(ctx, drops, p, gains=gains)
    bt.run()
    res = bt.results()
    bt.close()
    for d, r in zip(drops, res):
        parity.check_structure(d, r)
    op = oracle.Params(fixed_count=0)
    sample = np.random.default_rng(20240).choice(len(drops), 16, replace=False)
    diverged = 0
    for b in sample:
        d, r = drops[b], res[b]
        o = oracle.solve(d, op)
        info = parity.compare(d, r, o, label=f"benchmark drop {b}", allow_diverged=True)
        print(info, flush=True)
        diverged += bool(info.get("diverged"))
    assert diverged <= 1


def test_context_outlives_its_batches_and_networks():
    """Destroying a context while a batch and a network made on it are alive
    only closes it: they keep working, direct calls on the context are
    refused, and it is freed with the last of them."""
    import paper_1803_07772_amd as pa
    from paper_1803_07772_amd.mlp import MLP, init_params
    drops = _mixed_batch()[:3]
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=20)
    print("[gpu case] context closed before its batch and network", flush=True)
    c = pa.Context(0)
    ref = c.solve_batch(drops, p)
    bt = pa.Batch(c, drops, p)
    net = MLP(c, init_params(3))
    h = c._h
    c.close()
    held = pa.Context.__new__(pa.Context)  # a caller still holding the closed handle
    held._h = h
    with pytest.raises(pa.AllocError, match="-22"):
        held.solve(drops[0], p)
    held._h = None
    bt.run()
    for a, b in zip(bt.results(), ref):
        _same(a, b)
    net.solve(drops[0], p)
    bt.close()
    net.close()


def test_ragged_batch_full_size_against_stored_oracle(ctx):
    """The ragged 4096-drop batch (M-1 in 2..16, N in 64..1024, K in
    16..256, l = 3) in one graph launch, in the launch shape and schedule the
    benchmark times: the seeded 1% check subset (41 drops, the largest of
    them 3.85 M triples) element by element against the FP64 oracle's stored
    results, and every drop against what any allocation satisfies."""
    import torch

    import paper_1803_07772_amd as pa
    from paper_1803_07772_amd import tune
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "cfg4_subset.npz"))
    drops = synth.make_batch(4096, seed=0, threads=16)
    gains = [torch.from_numpy(d.gain).cuda() for d in drops]
    p = tune.tuned(drops, pa.Params(fixed_count=0))
    print(f"[gpu case] ragged 4096-drop batch, launch {p}", flush=True)
    bt = pa.Batch(ctx, drops, p, gains=gains)
    bt.run()
    res = bt.results()
    bt.close()
    del gains
    for d, r in zip(drops, res):
        parity.check_structure(d, r)
    assert not any(r.status_flags & pa.GROUP_TIMEOUT for r in res)
    flagged = 0
    for b in g["indices"].tolist():
        o = parity.load_stored(g, f"d{b}_", drops[b])
        info = parity.compare(drops[b], res[b], o, label=f"ragged drop {b} {drops[b].M}x{drops[b].N}x{drops[b].K}")
        flagged += info["flagged_mn"] + info["flagged_users"]
        print(info, flush=True)
    print("check subset: 41 drops at the bars, flagged elements", flagged, flush=True)
