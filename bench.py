"""Benchmark: allocations solved per second on one MI355X.

Workload (value): batches of drops of the 5-RRH, 64-subcarrier, 32-user
configuration (24 elastic, 8 streaming users, l=2), converge mode with caps,
solved by the batched persistent solver with the gains resident in HBM; one
step is one replay of the graph-captured batched solve of every drop, in the
launch shape the autotuner chose for the bucket.  Beside it, on the same GPU:
* batched_call: the same batch through one alloc_solve_batch call;
* cfg4_ragged: the first drops of the ragged 4096-drop batch (one graph
  replay; large drops split over several workgroups);
* plain: the same drops through alloc_solve, one after another;
* architectures: the paper's architecture comparison (H-CRAN with PD-NOMA,
  the same with one user per subcarrier, 1-tier C-RAN, 2-tier HCN, 1-tier
  HPN) on the same users under the paper's channel, one batch each;
* paper_sweeps (with --sweeps): the trend studies of the paper's simulation
  section (users, streaming users, arrival rate, PD-NOMA/OMA, LPN count);
* large_drop: the 17-RRH, 1024-subcarrier, 256-user drop (l=3, exactly 200
  sweeps per Dinkelbach step) through alloc_solve;
* nn_warm: a warm-start network trained on the GPU (solved drops of the same
  generator, other seeds), then network inference + warm-started batched
  solves of the benchmark's drops.
The roofline object is the dominant kernel's (the batched solver):
algorithmic bytes = 4 per (RRH, subcarrier, user) triple per sweep, over its
HIP-event duration.  The FP64 oracle is timed on a bounded sample of the same
drops on the host.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=4096, help="drops per step")
    ap.add_argument("--plain-drops", type=int, default=16)
    ap.add_argument("--train-drops", type=int, default=512)
    ap.add_argument("--train-steps", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-nn", action="store_true")
    ap.add_argument("--no-cfg4", action="store_true")
    ap.add_argument("--no-arch", action="store_true")
    ap.add_argument("--arch-drops", type=int, default=1024, help="drops per architecture")
    ap.add_argument("--sweeps", action="store_true",
                    help="also run the trend studies of the paper's simulation section")
    ap.add_argument("--sweep-drops", type=int, default=256, help="drops per point of --sweeps")
    ap.add_argument("--cfg4-drops", type=int, default=1024,
                    help="drops of the ragged 4096-drop batch timed in the cfg4 leg")
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


def counter_record(kernel: str, drops: int | None):
    """The committed counter summary of a kernel (profiles/traffic.json), if
    it was taken on the current kernel sources and the same batch size."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or drops is None:
        return None
    try:
        e = json.load(open(path))[kernel]
        if e["src_sha256"] != solver_source_sha() or e["drops_per_step"] != drops:
            return None
        return e
    except (KeyError, ValueError, OSError):
        return None


def traffic_for(kernel: str, drops: int | None):
    """HBM bytes per launch from the committed counter summary (else None)."""
    e = counter_record(kernel, drops)
    return e["hbm_bytes_per_launch"] if e else None


# Vector issue capacity: every wave64 VALU instruction holds its SIMD for at
# least 4 cycles; 256 CUs x 4 SIMDs at 2.4 GHz.
VALU_WAVE_INSTS_PEAK = 256 * 4 * 2.4e9 / 4


def valu_issue(kernel: str, drops: int | None, ms_per_launch: float):
    """VALU wave instructions per launch (rocprof SQ_INSTS_VALU, committed
    summary) against the vector issue capacity, or None."""
    e = counter_record(kernel, drops)
    if not e or "valu_wave_insts_per_launch" not in e:
        return None
    rate = e["valu_wave_insts_per_launch"] / (ms_per_launch * 1e-3)
    return {"wave_instructions_per_launch": e["valu_wave_insts_per_launch"], "achieved_per_s": rate,
            "peak_per_s": VALU_WAVE_INSTS_PEAK, "frac": rate / VALU_WAVE_INSTS_PEAK}


def roofline(kernel, bytes_per_launch, ms_per_launch, drops=None):
    ach = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(ach, 4), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": ach / HBM_PEAK_GBS, "traffic": traffic_for(kernel, drops), "kernel": kernel,
         "algorithmic_bytes_per_launch": bytes_per_launch, "ms_per_launch": ms_per_launch}
    v = valu_issue(kernel, drops, ms_per_launch)
    if v:
        r["valu_issue"] = v
    return r


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
             "qos_infeasible": int(sum(bool(r.status_flags & 2) for r in rs))})
    out["drops_per_point"] = drops_per_point
    out["allocations_per_s"] = solved / t_solve
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported: drops would shard "
              "across GPUs with no exchange, and only the one-GPU path is run and reported.", flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1803_07772_amd as pa
    import synth

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
    drops = [synth.make_drop(synth.CFG2, s, 0) for s in range(a.batch)]
    gains = [torch.from_numpy(d.gain).to(dev) for d in drops]
    torch.cuda.synchronize()
    print(f"[bench] {a.batch} drops of M=5 N=64 K=32 resident; warmup {a.warmup}, steps {a.steps}",
          flush=True)

    # launch shape: the autotuner's cached choice for this size bucket, or
    # measured now on a sample of the batch
    from paper_1803_07772_amd import tune
    cache = tune.load_cache()
    key = tune.batch_key(drops)
    if key in cache and not a.save_tune:
        params_b, tuned_from = tune.tuned(drops, params, cache), "cache"
    else:
        best, _ = tune.tune(ctx, drops, params, gains=gains, cache=cache)
        params_b, tuned_from = dataclasses.replace(params, **best), "measured"
    print(f"[bench] launch shape {key}: lds_kb={params_b.lds_kb} tile={params_b.tile} block={params_b.block or 512} wave={params_b.wave} "
          f"({tuned_from})", flush=True)

    # one step = one replay of the graph-captured batched solve of all drops
    bt = pa.Batch(ctx, drops, params_b, gains=gains)
    for _ in range(a.warmup):
        bt.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms_runs = []
    for _ in range(a.steps):
        bt.run()
        kms_runs.append(bt.last_ms())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] batched: {dt / a.steps * 1e3:.1f} ms per step", flush=True)
    value = a.batch * a.steps / dt
    kms = float(np.mean(kms_runs))
    res0 = bt.results()
    bt.close()
    bytes_launch = float(sum(4.0 * d.M * d.N * d.K * r.sweeps for d, r in zip(drops, res0)))
    line = {
        "metric": METRIC, "value": value, "unit": "allocations/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generator: 3GPP-style path loss, shadowing, Rayleigh)",
        "config": {"workload": "batched solver, drops of M=5 N=64 K=32 (24 elastic, 8 streaming) l=2, "
                               "converge with caps", "drops_per_step": a.batch, "mode": "batched",
                   "launch": {"graph": True, "lds_kb": params_b.lds_kb, "tile": params_b.tile,
                              "block": params_b.block or 512, "wave": params_b.wave, "tuned_from": tuned_from, "bucket": key}},
        "roofline": roofline("batch_kernel", bytes_launch, kms, a.batch),
        "sweeps_mean": float(np.mean([r.sweeps for r in res0])),
        "ee_mean": float(np.mean([r.ee for r in res0])),
    }
    modes = {"batched": {"allocations_per_s": value, "kernel_ms": kms, "graph": True}}
    t0 = time.perf_counter()
    ctx.solve_batch(drops, params_b, gains=gains)
    modes["batched_call"] = {"allocations_per_s": a.batch / (time.perf_counter() - t0),
                             "note": "one alloc_solve_batch call (descriptors uploaded, results copied back)"}

    if not a.no_cfg4:
        # the ragged batch (M-1 LPNs uniform in 2..16, N in {64..1024}, K in
        # 16..256, a quarter streaming): the first cfg4_drops of its 4096 drops
        d4 = synth.make_batch(4096, seed=0)[:a.cfg4_drops]
        g4 = [torch.from_numpy(d.gain).to(dev) for d in d4]
        k4 = tune.batch_key(d4)
        if k4 in cache and not a.save_tune:
            p4, t4 = tune.tuned(d4, params, cache), "cache"
        else:
            best4, _ = tune.tune(ctx, d4, params, gains=g4, cache=cache)
            p4, t4 = dataclasses.replace(params, **best4), "measured"
        b4 = pa.Batch(ctx, d4, p4, gains=g4)
        t0 = time.perf_counter()
        b4.run()
        dt4 = time.perf_counter() - t0
        r4 = b4.results()
        ms4 = b4.last_ms()
        b4.close()
        by4 = float(sum(4.0 * d.M * d.N * d.K * r.sweeps for d, r in zip(d4, r4)))
        modes["cfg4_ragged"] = {
            "workload": f"first {len(d4)} drops of the ragged 4096-drop batch (seed 0), one graph replay",
            "allocations_per_s": len(d4) / dt4, "triples": int(sum(d.M * d.N * d.K for d in d4)),
            "sweeps_mean": float(np.mean([r.sweeps for r in r4])),
            "groups_timeout": int(sum(bool(r.status_flags & 32) for r in r4)),
            "launch": {"lds_kb": p4.lds_kb, "tile": p4.tile, "block": p4.block or 512, "wave": p4.wave, "tuned_from": t4,
                       "bucket": k4},
            "roofline": roofline("batch_kernel", by4, ms4)}
        del g4
        print(f"[bench] cfg4 ragged: {len(d4) / dt4:.1f} allocations/s", flush=True)
    if a.save_tune:
        tune.save_cache(cache, a.save_tune)
        print(f"[bench] saved the autotuner cache ({len(cache)} buckets)", flush=True)

    if not a.no_plain:
        sub = list(zip(drops, gains))[:a.plain_drops]
        for d, g in sub[:2]:
            ctx.solve(d, params, gain=g)
        rs = []
        t0 = time.perf_counter()
        for d, g in sub:
            r = ctx.solve(d, params, gain=g)
            rs.append((d, r, ctx.last_kernel_ms()))
        dtp = time.perf_counter() - t0
        b = float(np.mean([4.0 * d.M * d.N * d.K * r.sweeps for d, r, _ in rs]))
        modes["plain"] = {"allocations_per_s": len(sub) / dtp, "drops": len(sub),
                          "roofline": roofline("solve_kernel", b, float(np.mean([k for _, _, k in rs])))}
        print(f"[bench] plain: {len(sub) / dtp:.1f} allocations/s", flush=True)

    if not a.no_arch:
        # the architecture comparison of the paper's simulation section: the
        # same users and fading under the paper's channel, solved as one
        # batch per architecture
        arch = {}
        for kind in synth.ARCHITECTURES:
            da = [synth.architecture_drop(kind, 0, i) for i in range(a.arch_drops)]
            ga = [torch.from_numpy(d.gain).to(dev) for d in da]
            ka = tune.batch_key(da)
            if a.save_tune:
                best_a, _ = tune.tune(ctx, da, params, gains=ga, cache=cache)
                pk, tk = dataclasses.replace(params, **best_a), "measured"
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
                          "qos_infeasible": int(sum(bool(r.status_flags & pa.QOS_INFEASIBLE) for r in ra)),
                          "launch": {"lds_kb": pk.lds_kb, "tile": pk.tile, "block": pk.block or 512,
                                     "wave": pk.wave, "tuned_from": tk, "bucket": ka}}
            del ga
        base = arch["hcran"]["ee_mean"]
        for kind in arch:
            arch[kind]["ee_over_hcran"] = arch[kind]["ee_mean"] / base
        modes["architectures"] = {
            "workload": f"{a.arch_drops} drops per architecture of the paper's channel "
                        "(chi d^-3, 42/23 dBm, N=32, K=12 of which 6 streaming at 125 packets/s), "
                        "one graph replay each", **arch}
        print("[bench] architectures: " + ", ".join(f"{k} EE {v['ee_mean']:.1f}" for k, v in arch.items()),
              flush=True)

    if a.save_tune and not a.no_arch:
        tune.save_cache(cache, a.save_tune)

    if a.sweeps:
        modes["paper_sweeps"] = paper_sweeps(ctx, params, a.sweep_drops)
        print("[bench] paper sweeps done", flush=True)

    if not a.no_large:
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
                               "roofline": roofline("solve_kernel", b, float(np.mean([k for _, k in rs])))}
        print(f"[bench] large drop: {dt3 * 1e3:.1f} ms per solve", flush=True)

    if not a.no_nn:
        from paper_1803_07772_amd import warm
        tdrops = [synth.make_drop(synth.CFG2, 1_000_000 + s, 0) for s in range(a.train_drops)]
        tg = [torch.from_numpy(d.gain).to(dev) for d in tdrops]
        cfg = warm.TrainConfig(steps=a.train_steps)
        net, info = warm.fit(ctx, tdrops, params, cfg, gains=tg)
        print(f"[bench] trained: {info}", flush=True)
        net.solve_batch(drops[:64], params_b, gains=gains[:64])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wr = net.solve_batch(drops, params_b, gains=gains)
        dtw = time.perf_counter() - t0
        mlp_ms = net.last_ms()
        rows = sum(d.M * d.N * d.K for d in drops)
        tfl = MLP_FLOP_PER_ROW * rows / (mlp_ms * 1e-3) / 1e12
        ee_ratio = np.array([w.ee / c.ee for w, c in zip(wr, res0)])
        modes["nn_warm"] = {
            "allocations_per_s": a.batch / dtw, "includes": "network inference + warm-started batched solve",
            "train": {k: v for k, v in info.items()}, "train_drops": a.train_drops,
            "sweeps_mean_warm": float(np.mean([r.sweeps for r in wr])),
            "sweeps_mean_cold": line["sweeps_mean"],
            "ee_ratio_warm_over_cold_mean": float(ee_ratio.mean()),
            "ee_ratio_min": float(ee_ratio.min()),
            "fallbacks": int(sum(bool(r.status_flags & pa.WARM_FALLBACK) for r in wr)),
            "mlp_ms": mlp_ms,
            "mlp_roofline": {"bound": "mfma", "achieved": tfl, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": tfl / BF16_PEAK_TFLOPS, "flop_per_row": MLP_FLOP_PER_ROW, "rows": rows},
        }
        print(f"[bench] nn warm: {a.batch / dtw:.1f} allocations/s", flush=True)
    line["modes"] = modes

    if not a.no_cpu_baseline:
        import oracle
        op = oracle.Params(fixed_count=0)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < 10.0:
            oracle.solve(drops[n % len(drops)], op)
            n += 1
        dtc = time.perf_counter() - t0
        cores = oracle.set_threads(1)
        t1 = time.perf_counter()
        n1 = 0
        while time.perf_counter() - t1 < 5.0:
            oracle.solve(drops[n1 % len(drops)], op)
            n1 += 1
        dt1 = time.perf_counter() - t1
        oracle.set_threads(cores)
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
        except OSError:
            pass
        line["cpu_baseline"] = {"value": n / dtc, "unit": "allocations/s", "cores": cores,
                                "kind": "oracle",
                                "sample": f"{n} solves of the first drops of the benchmark batch in "
                                          f"{dtc:.1f} s (FP64 C oracle, OpenMP over subcarriers)",
                                "single_thread": {"value": n1 / dt1, "solves": n1, "seconds": dt1},
                                "cpu_model": model}
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
