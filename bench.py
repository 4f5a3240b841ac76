"""Benchmark: allocations solved per second on one MI355X.

Workload (value): the ragged batch of 4096 independent drops (M - 1 LPNs
uniform in 2..16, N uniform in {64, 128, 256, 512, 1024}, K uniform in
16..256 with a quarter streaming, l = 3; seeded synthetic channels), solved
by the batched persistent solver in one graph-captured launch per step, in
converge mode with caps, gains resident in HBM, in the launch shape and
schedule the autotuner chose for the batch.  The value counts only when the
accuracy gate passes: the 41 drops of the check subset (a seeded 1%) are
compared element by element with the FP64 oracle's stored results (EE within
1e-5 relative, assignments and decoding orders identical and powers within
1e-4 relative wherever the oracle flagged no near-tie).

Beside it, on the same GPU (each within the time budget left after the
headline; a leg that does not fit is recorded as skipped):
* cfg2_batched: 4096 drops of 5 RRHs x 64 subcarriers x 32 users, one graph
  replay, and the same batch through one alloc_solve_batch call;
* plain: drops of that configuration through alloc_solve, one per launch;
* large_drop: the 17-RRH, 1024-subcarrier, 256-user drop (l = 3, exactly
  200 sweeps per Dinkelbach step) through alloc_solve;
* nn_warm: the warm-start network trained on the GPU on drops of the
  17 x 1024 x 256 generator (subsampled triples), then inference plus
  warm-started batched solves of fresh drops of that generator against their
  cold solves (dual sweeps, EE ratio, fallbacks);
* architectures: the paper's architecture comparison on its channel;
* paper_sweeps (with --sweeps): the trend studies of the simulation section.
The roofline object is the dominant kernel's (the batched solver):
algorithmic bytes = 4 per (RRH, subcarrier, user) triple per sweep, over its
HIP-event duration.  The FP64 oracle is timed on a bounded sample of the
headline workload's drops on the host.
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
MLP_FLOP_PER_ROW = 2 * (4 * 256 + 256 * 256 + 256 * 256 + 256 * 3)
METRIC = "allocations solved/s at ≤1e-5 rel EE error; plain vs batched vs NN warm start"
GATE_PATH = os.path.join(ROOT, "tests", "golden", "cfg4_subset.npz")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=4096, help="drops of the ragged batch")
    ap.add_argument("--budget-s", type=float, default=540.0,
                    help="wall-clock budget of the whole run: legs after the headline run while "
                         "their estimated time fits")
    ap.add_argument("--plain-drops", type=int, default=16)
    ap.add_argument("--train-drops", type=int, default=128,
                    help="drops of the 17 x 1024 x 256 generator the network is trained on")
    ap.add_argument("--eval-drops", type=int, default=64,
                    help="fresh drops of that generator the warm start is evaluated on")
    ap.add_argument("--train-steps", type=int, default=300)
    ap.add_argument("--warm-cap", type=int, default=4,
                    help="Dinkelbach steps of the warm-started attempt before it falls back to the cold solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-nn", action="store_true")
    ap.add_argument("--no-cfg2", action="store_true")
    ap.add_argument("--no-arch", action="store_true")
    ap.add_argument("--arch-drops", type=int, default=1024, help="drops per architecture")
    ap.add_argument("--sweeps", action="store_true",
                    help="also run the trend studies of the paper's simulation section")
    ap.add_argument("--sweep-drops", type=int, default=256, help="drops per point of --sweeps")
    ap.add_argument("--save-tune", metavar="PATH", default=None,
                    help="run the autotuner for every workload here and save its cache to PATH")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 256 MiB device to device three times (a kernel of known "
                         "traffic, for scaling memory counters)")
    return ap.parse_args()


def solver_source_sha() -> str:
    """sha256 over the solver kernel's sources (alloc.hip and the headers it
    includes), in a fixed order."""
    h = hashlib.sha256()
    for f in ("alloc.hip", "ctx.h", "logs.h"):
        h.update(open(os.path.join(ROOT, "paper_1803_07772_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def counter_record(kernel: str, workload: str | None):
    """The committed counter summary of a kernel (profiles/traffic.json), if
    it was taken on the current kernel sources and the same workload."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or workload is None:
        return None
    try:
        e = json.load(open(path))[kernel]
        if e["src_sha256"] != solver_source_sha() or e["workload"] != workload:
            return None
        return e
    except (KeyError, ValueError, OSError):
        return None


def traffic_for(kernel: str, workload: str | None):
    """HBM bytes per launch from the committed counter summary (else None)."""
    e = counter_record(kernel, workload)
    return e["hbm_bytes_per_launch"] if e else None


# Vector issue capacity: every wave64 VALU instruction holds its SIMD for at
# least 4 cycles; 256 CUs x 4 SIMDs at 2.4 GHz.
VALU_WAVE_INSTS_PEAK = 256 * 4 * 2.4e9 / 4


def valu_issue(kernel: str, workload: str | None, ms_per_launch: float):
    """VALU wave instructions per launch (rocprof SQ_INSTS_VALU, committed
    summary) against the vector issue capacity, or None."""
    e = counter_record(kernel, workload)
    if not e or "valu_wave_insts_per_launch" not in e:
        return None
    rate = e["valu_wave_insts_per_launch"] / (ms_per_launch * 1e-3)
    return {"wave_instructions_per_launch": e["valu_wave_insts_per_launch"], "achieved_per_s": rate,
            "peak_per_s": VALU_WAVE_INSTS_PEAK, "frac": rate / VALU_WAVE_INSTS_PEAK}


def roofline(kernel, bytes_per_launch, ms_per_launch, workload=None):
    ach = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(ach, 4), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": ach / HBM_PEAK_GBS, "traffic": traffic_for(kernel, workload), "kernel": kernel,
         "algorithmic_bytes_per_launch": bytes_per_launch, "ms_per_launch": ms_per_launch}
    v = valu_issue(kernel, workload, ms_per_launch)
    if v:
        r["valu_issue"] = v
    return r


def algorithmic_bytes(drops, results) -> float:
    """4 bytes (one float32 gain read) per triple per sweep."""
    return float(sum(4.0 * d.M * d.N * d.K * r.sweeps for d, r in zip(drops, results)))


def gate(drops, results, path=GATE_PATH):
    """The accuracy gate: the check subset's drops against the oracle's
    stored results, at the parity bars of tests/parity.py (EE within 1e-5
    relative; assignments, decoding orders and powers on every element the
    oracle did not flag).  Returns {checked, passed, failed: [...]}."""
    import numpy as np

    from tests import parity
    g = np.load(path)
    out = {"checked": 0, "passed": 0, "failed": [], "flagged_elements": 0,
           "subset": "41 drops (1%) of the batch by a seeded permutation; "
                     "stored FP64 oracle results (tests/golden/cfg4_subset.npz)"}
    for b in g["indices"].tolist():
        d, r = drops[b], results[b]
        o = parity.load_stored(g, f"d{b}_", d)
        out["checked"] += 1
        try:
            info = parity.compare(d, r, o, label=f"drop {b}")
            out["passed"] += 1
            out["flagged_elements"] += info["flagged_mn"] + info["flagged_users"]
        except AssertionError as e:
            out["failed"].append({"drop": b, "detail": str(e)[:300]})
    return out


def paper_sweeps(ctx, params, drops_per_point: int):
    """The trend studies of the paper's simulation section on its channel:
    EE of the elastic users against the number of users for several counts of
    streaming users, for several packet arrival rates, and with PD-NOMA
    against OMA; and against the number of LPN RRHs (12 users, half
    streaming).  One batched solve of drops_per_point drops per point."""
    import dataclasses as dc

    import numpy as np

    import synth
    base = synth.PAPER
    pts = []
    for ks in (2, 4, 6):
        for k in (8, 12, 16, 20, 24, 28):
            pts.append(("streaming_users", dict(K_s=ks), k, dc.replace(base, K=k, K_s=ks)))
    for lam in (62.5, 125.0, 250.0):
        for k in (12, 16, 20, 24, 28):
            rate = lam * base.packet_bits
            pts.append(("arrival_rate", dict(packets_per_s=lam), k,
                        dc.replace(base, K=k, K_s=6, rate_bps_lo=rate, rate_bps_hi=rate)))
    for l in (2, 1):
        for k in (12, 16, 20, 24, 28):
            pts.append(("noma_vs_oma", dict(l=l), k, dc.replace(base, K=k, K_s=6, l=l)))
        for mf in (1, 2, 3, 4, 5, 6):
            pts.append(("lpn_count", dict(l=l), mf, dc.replace(base, M=1 + mf, K=12, K_s=6, l=l)))
    out, solved, t_solve = {}, 0, 0.0
    for study, series, x, rc in pts:
        drops = [synth.make_drop(rc, 0, i) for i in range(drops_per_point)]
        t0 = time.perf_counter()
        rs = ctx.solve_batch(drops, params)
        t_solve += time.perf_counter() - t0
        solved += len(drops)
        key = ",".join(f"{a}={b}" for a, b in series.items())
        out.setdefault(study, {}).setdefault(key, []).append(
            {"x": x, "ee_mean": float(np.mean([r.ee for r in rs])),
             "infeasible": {f: int(sum(bool(r.status_flags & v) for r in rs))
                            for f, v in (("qos", 2), ("sic", 16), ("budget", 64))}})
    out["drops_per_point"] = drops_per_point
    out["allocations_per_s"] = solved / t_solve
    return out


def flag_counts(results):
    import paper_1803_07772_amd as pa
    return {name: int(sum(bool(r.status_flags & v) for r in results))
            for name, v in (("not_converged", pa.NOT_CONVERGED), ("qos_infeasible", pa.QOS_INFEASIBLE),
                            ("sic_infeasible", pa.SIC_INFEASIBLE), ("budget_infeasible", pa.BUDGET_INFEASIBLE),
                            ("nonfinite", pa.NONFINITE), ("group_timeout", pa.GROUP_TIMEOUT))}


def launch_of(p, tuned_from, key):
    return {"graph": True, "lds_kb": p.lds_kb, "tile": p.tile, "block": p.block or 512, "wave": p.wave,
            "group_triples": p.group_triples, "tuned_from": tuned_from, "bucket": key}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported: drops would shard "
              "across GPUs with no exchange, and only the one-GPU path is run and reported.", flush=True)
        sys.exit(2)
    t_start = time.perf_counter()
    import numpy as np
    import torch

    import paper_1803_07772_amd as pa
    import synth
    from paper_1803_07772_amd import tune

    def left():
        return a.budget_s - (time.perf_counter() - t_start)

    dev = torch.device("cuda:0")
    if a.calibrate_copy:
        src = torch.ones(1 << 26, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = pa.Context(0)
    ctx.set_timing(True)
    params = pa.Params(fixed_count=0)  # converge with caps: 200 sweeps per step, 20 steps
    threads = min(16, os.cpu_count() or 1)
    drops = synth.make_batch(a.batch, seed=0, threads=threads)
    gains = [torch.from_numpy(d.gain).to(dev) for d in drops]
    torch.cuda.synchronize()
    triples = int(sum(d.M * d.N * d.K for d in drops))
    print(f"[bench] ragged batch of {a.batch} drops ({triples / 1e9:.2f} G triples) resident; "
          f"warmup {a.warmup}, steps {a.steps}", flush=True)

    # launch shape and schedule: the autotuner's cached choice for the
    # batch's bucket, or measured now
    cache = tune.load_cache()
    key = tune.batch_key(drops)
    if key in cache and not a.save_tune:
        p4, tuned_from = tune.tuned(drops, params, cache), "cache"
    else:
        best, _ = tune.tune(ctx, drops, params, gains=gains, cache=cache)
        p4, tuned_from = dataclasses.replace(params, **best), "measured"
    print(f"[bench] launch {key}: {launch_of(p4, tuned_from, key)}", flush=True)

    # one step = one replay of the graph-captured batched solve of all drops
    bt = pa.Batch(ctx, drops, p4, gains=gains)
    for _ in range(a.warmup):
        bt.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms_runs = []
    for s in range(a.steps):
        bt.run()
        kms_runs.append(bt.last_ms())
        print(f"[bench] step {s}: {kms_runs[-1]:.1f} ms", flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = bt.results()
    bt.close()
    kms = float(np.mean(kms_runs))
    measured = a.batch * a.steps / dt
    g = gate(drops, res) if a.batch == 4096 else {"checked": 0, "passed": 0, "failed": [],
                                                 "note": "the check subset belongs to the 4096-drop batch"}
    gate_ok = g["checked"] > 0 and g["passed"] == g["checked"]
    print(f"[bench] ragged batch: {dt / a.steps * 1e3:.1f} ms per step, {measured:.1f} allocations/s; "
          f"gate {g['passed']}/{g['checked']}", flush=True)
    workload = (f"ragged batch of {a.batch} drops (M-1 in 2..16, N in 64..1024, K in 16..256, "
                "a quarter streaming, l=3, seed 0), one persistent graph-captured launch, converge with caps")
    sweeps = np.array([r.sweeps for r in res])
    line = {
        "metric": METRIC, "value": measured if gate_ok else 0.0, "unit": "allocations/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generator: 3GPP-style path loss, shadowing, Rayleigh)",
        "config": {"workload": workload, "drops_per_step": a.batch, "triples": triples, "mode": "batched",
                   "launch": launch_of(p4, tuned_from, key)},
        "gate": g,
        "roofline": roofline("batch_kernel", algorithmic_bytes(drops, res), kms, "cfg4"),
        "sweeps_mean": float(sweeps.mean()), "sweeps_max": int(sweeps.max()),
        "ee_mean": float(np.mean([r.ee for r in res])),
        "flags": flag_counts(res),
    }
    if not gate_ok:
        line["measured_before_gate"] = measured
    modes = {"ragged_batched": {"allocations_per_s": measured, "kernel_ms": kms, "graph": True}}
    del gains
    torch.cuda.empty_cache()

    if not a.no_cfg2 and left() > 60:
        d2 = [synth.make_drop(synth.CFG2, s, 0) for s in range(4096)]
        g2 = [torch.from_numpy(d.gain).to(dev) for d in d2]
        k2 = tune.batch_key(d2)
        if k2 in cache and not a.save_tune:
            p2, t2 = tune.tuned(d2, params, cache), "cache"
        else:
            best2, _ = tune.tune(ctx, d2, params, gains=g2, cache=cache)
            p2, t2 = dataclasses.replace(params, **best2), "measured"
        b2 = pa.Batch(ctx, d2, p2, gains=g2)
        b2.run()
        ms2 = []
        for _ in range(3):
            b2.run()
            ms2.append(b2.last_ms())
        r2 = b2.results()
        b2.close()
        t0 = time.perf_counter()
        ctx.solve_batch(d2, p2, gains=g2)
        call = len(d2) / (time.perf_counter() - t0)
        ms2m = float(np.mean(ms2))
        modes["cfg2_batched"] = {
            "workload": "4096 drops of M=5 N=64 K=32 (24 elastic, 8 streaming) l=2, one graph replay",
            "allocations_per_s": len(d2) / (ms2m * 1e-3), "kernel_ms": ms2m,
            "one_call_allocations_per_s": call,
            "sweeps_mean": float(np.mean([r.sweeps for r in r2])), "flags": flag_counts(r2),
            "launch": launch_of(p2, t2, k2),
            "roofline": roofline("batch_kernel", algorithmic_bytes(d2, r2), ms2m, "cfg2")}
        print(f"[bench] cfg2 batched: {len(d2) / (ms2m * 1e-3):.1f} allocations/s", flush=True)

        if not a.no_plain and left() > 30:
            sub = list(zip(d2, g2))[:a.plain_drops]
            for d, gg in sub[:2]:
                ctx.solve(d, params, gain=gg)
            rs = []
            t0 = time.perf_counter()
            for d, gg in sub:
                r = ctx.solve(d, params, gain=gg)
                rs.append((d, r, ctx.last_kernel_ms()))
            dtp = time.perf_counter() - t0
            b = float(np.mean([4.0 * d.M * d.N * d.K * r.sweeps for d, r, _ in rs]))
            modes["plain"] = {"workload": "drops of M=5 N=64 K=32 through alloc_solve, one per launch",
                              "allocations_per_s": len(sub) / dtp, "drops": len(sub),
                              "roofline": roofline("solve_kernel", b, float(np.mean([k for _, _, k in rs])))}
            print(f"[bench] plain: {len(sub) / dtp:.1f} allocations/s", flush=True)
        del g2
    if a.save_tune:
        tune.save_cache(cache, a.save_tune)
        print(f"[bench] saved the autotuner cache ({len(cache)} buckets)", flush=True)

    if not a.no_large and left() > 30:
        d3 = synth.make_drop(synth.CFG3, 0, 0)
        g3 = torch.from_numpy(d3.gain).to(dev)
        p3 = pa.Params()  # exactly 200 sweeps per Dinkelbach step
        ctx.solve(d3, p3, gain=g3)
        rs = []
        t0 = time.perf_counter()
        for _ in range(3):
            r = ctx.solve(d3, p3, gain=g3)
            rs.append((r, ctx.last_kernel_ms()))
        dt3 = (time.perf_counter() - t0) / 3
        b = 4.0 * d3.M * d3.N * d3.K * rs[-1][0].sweeps
        modes["large_drop"] = {"workload": "M=17 N=1024 K=256 l=3, 200 sweeps per Dinkelbach step",
                               "allocations_per_s": 1.0 / dt3, "ms_per_solve": dt3 * 1e3,
                               "sweeps": rs[-1][0].sweeps, "ee": rs[-1][0].ee,
                               "status_flags": rs[-1][0].status_flags,
                               "roofline": roofline("solve_kernel", b, float(np.mean([k for _, k in rs])))}
        print(f"[bench] large drop: {dt3 * 1e3:.1f} ms per solve", flush=True)
        del g3

    if not a.no_nn and left() > 90:
        modes["nn_warm"] = nn_warm(a, ctx, params, dev)

    if not a.no_arch and left() > 45:
        modes["architectures"] = architectures(a, ctx, params, dev, cache)

    if a.sweeps and left() > 60:
        modes["paper_sweeps"] = paper_sweeps(ctx, params, a.sweep_drops)
        print("[bench] paper sweeps done", flush=True)
    skipped = [m for m, off in (("cfg2_batched", a.no_cfg2), ("large_drop", a.no_large), ("nn_warm", a.no_nn),
                                ("architectures", a.no_arch)) if not off and m not in modes]
    if skipped:
        line["skipped_for_time"] = skipped
    line["modes"] = modes

    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(drops, res, max(5.0, min(20.0, left() - 5.0)))
    ctx.close()
    line["wall_s"] = time.perf_counter() - t_start
    print(json.dumps(line), flush=True)


def nn_warm(a, ctx, params, dev):
    """The warm-start network on the 17 x 1024 x 256 generator: trained on
    a.train_drops drops solved cold (2048 sampled triples per drop), then
    evaluated on a.eval_drops fresh drops: network inference + warm-started
    batched solve against the cold batched solve of the same drops."""
    import numpy as np
    import torch

    import paper_1803_07772_amd as pa
    import synth
    from paper_1803_07772_amd import warm
    tdrops = [synth.make_drop(synth.CFG3, 1 + s, 0) for s in range(a.train_drops)]
    tg = [torch.from_numpy(d.gain).to(dev) for d in tdrops]
    net, info = warm.fit(ctx, tdrops, params, warm.TrainConfig(steps=a.train_steps), gains=tg, chunk=32)
    del tg
    print(f"[bench] trained: {info}", flush=True)
    edrops = [synth.make_drop(synth.CFG3, 1_000_000 + s, 0) for s in range(a.eval_drops)]
    eg = [torch.from_numpy(d.gain).to(dev) for d in edrops]
    wparams = dataclasses.replace(params, warm_max_dinkelbach=a.warm_cap)
    net.solve_batch(edrops[:2], wparams, gains=eg[:2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cold = ctx.solve_batch(edrops, params, gains=eg)
    dtc = time.perf_counter() - t0
    t0 = time.perf_counter()
    wr = net.solve_batch(edrops, wparams, gains=eg)
    dtw = time.perf_counter() - t0
    mlp_ms = net.last_ms()
    rows = sum(d.M * d.N * d.K for d in edrops)
    tfl = MLP_FLOP_PER_ROW * rows / (mlp_ms * 1e-3) / 1e12
    ratio = np.array([w.ee / c.ee for w, c in zip(wr, cold)])
    net.close()
    out = {
        "workload": f"trained on {a.train_drops} drops of the M=17 N=1024 K=256 generator (seeds 1..), "
                    f"evaluated on {a.eval_drops} fresh drops (seeds 1000000..); a fraction of the "
                    "200k-drop training set and 4096 evaluation drops",
        "allocations_per_s": a.eval_drops / dtw, "cold_allocations_per_s": a.eval_drops / dtc,
        "includes": "network inference + warm-started batched solve (one alloc_solve_batch_mlp call), "
                    f"at most {a.warm_cap} Dinkelbach steps for the warm attempt, then the cold fallbacks",
        "train": info, "sweeps_mean_warm": float(np.mean([r.sweeps for r in wr])),
        "sweeps_mean_cold": float(np.mean([r.sweeps for r in cold])),
        "dinkelbach_mean_warm": float(np.mean([r.dinkelbach_iters for r in wr])),
        "dinkelbach_mean_cold": float(np.mean([r.dinkelbach_iters for r in cold])),
        "ee_ratio_warm_over_cold_mean": float(ratio.mean()), "ee_ratio_min": float(ratio.min()),
        "ee_ratio_q05": float(np.quantile(ratio, 0.05)),
        "fallbacks": int(sum(bool(r.status_flags & pa.WARM_FALLBACK) for r in wr)),
        "flags_warm": flag_counts(wr), "flags_cold": flag_counts(cold),
        "mlp_ms": mlp_ms,
        "mlp_roofline": {"bound": "mfma", "achieved": tfl, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tfl / BF16_PEAK_TFLOPS, "flop_per_row": MLP_FLOP_PER_ROW, "rows": rows},
    }
    print(f"[bench] nn warm: {a.eval_drops / dtw:.2f} allocations/s (cold {a.eval_drops / dtc:.2f}); "
          f"sweeps {out['sweeps_mean_warm']:.0f} vs {out['sweeps_mean_cold']:.0f}", flush=True)
    return out


def architectures(a, ctx, params, dev, cache):
    """The architecture comparison of the paper's simulation section: the
    same users and fading under the paper's channel, one batch each."""
    import numpy as np
    import torch

    import paper_1803_07772_amd as pa
    import synth
    from paper_1803_07772_amd import tune
    arch = {}
    for kind in synth.ARCHITECTURES:
        da = [synth.architecture_drop(kind, 0, i) for i in range(a.arch_drops)]
        ga = [torch.from_numpy(d.gain).to(dev) for d in da]
        ka = tune.batch_key(da)
        if a.save_tune:
            best_a, _ = tune.tune(ctx, da, params, gains=ga, cache=cache)
            pk, tk = dataclasses.replace(params, **best_a), "measured"
            tune.save_cache(cache, a.save_tune)
        elif ka in cache:
            pk, tk = tune.tuned(da, params, cache), "cache"
        else:  # untuned bucket: the default launch shape
            pk, tk = params, "default"
        ba = pa.Batch(ctx, da, pk, gains=ga)
        ba.run()
        ba.run()
        msa = ba.last_ms()
        ra = ba.results()
        ba.close()
        ee = np.array([r.ee for r in ra])
        arch[kind] = {"allocations_per_s": len(da) / (msa * 1e-3), "kernel_ms": msa,
                      "M": da[0].M, "l": da[0].l, "ee_mean": float(ee.mean()),
                      "ee_median": float(np.median(ee)),
                      "rate_sum_mean": float(np.mean([r.rate_sum for r in ra])),
                      "power_sum_mean": float(np.mean([r.power_sum for r in ra])),
                      "sweeps_mean": float(np.mean([r.sweeps for r in ra])),
                      "flags": flag_counts(ra), "launch": launch_of(pk, tk, ka)}
        del ga
    base = arch["hcran"]["ee_mean"]
    for kind in arch:
        arch[kind]["ee_over_hcran"] = arch[kind]["ee_mean"] / base
    print("[bench] architectures: " + ", ".join(f"{k} EE {v['ee_mean']:.1f}" for k, v in arch.items()),
          flush=True)
    return {"workload": f"{a.arch_drops} drops per architecture of the paper's channel "
                        "(chi d^-3, 42/23 dBm, N=32, K=12 of which 6 streaming at 125 packets/s), "
                        "one graph replay each", **arch}


def cpu_baseline(drops, results, seconds):
    """The FP64 oracle on the host cores: the headline batch's drops in a
    seeded order for about `seconds`; allocations/s of that sample, and
    scaled to the batch's mix by the work (triples x sweeps) of the sample
    against the batch's mean.  Then the same on one thread."""
    import numpy as np

    import oracle
    order = np.random.default_rng(4).permutation(len(drops))
    op = oracle.Params(fixed_count=0)
    mean_work = float(np.mean([d.M * d.N * d.K * r.sweeps for d, r in zip(drops, results)]))

    def run(limit):
        t0 = time.perf_counter()
        n = work = 0
        while n < len(order) and time.perf_counter() - t0 < limit:
            d = drops[int(order[n])]
            r = oracle.solve(d, op)
            work += d.M * d.N * d.K * r.sweeps
            n += 1
        dt = time.perf_counter() - t0
        return n, dt, work

    n, dtc, work = run(seconds)
    cores = oracle.set_threads(1)
    n1, dt1, work1 = run(max(3.0, seconds / 3))
    oracle.set_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": (work / dtc) / mean_work, "unit": "allocations/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} solves of drops of the ragged batch in seeded order in {dtc:.1f} s "
                      f"({n / dtc:.2f} of those drops/s; value scaled to the batch's mean work of "
                      f"{mean_work:.3g} triple-sweeps per drop); FP64 C oracle, OpenMP over subcarriers",
            "sample_allocations_per_s": n / dtc, "sample_work_triple_sweeps": work,
            "single_thread": {"value": (work1 / dt1) / mean_work, "solves": n1, "seconds": dt1},
            "cpu_model": model}


if __name__ == "__main__":
    main()
