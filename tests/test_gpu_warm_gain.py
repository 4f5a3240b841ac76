"""What the trained warm-start network gains over the cold start.

A network is trained on the GPU (its own forward/backward kernels and AdamW)
on drops of the 5-RRH / 64-subcarrier / 32-user generator solved cold by the
batched solver, then held-out drops of the same generator are solved cold and
warm-started.  The warm start must save dual sweeps on average while the
energy efficiency it reaches stays that of the cold start on the typical
drop (the method is a local one: single drops may settle elsewhere, so the
median and the mean are bounded, not the minimum).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_trained_warm_start_saves_sweeps():
    import torch

    import paper_1803_07772_amd as pa
    from paper_1803_07772_amd import warm
    from paper_1803_07772_amd.mlp import MLP, init_params
    assert torch.cuda.is_available()
    ctx = pa.Context(0)
    params = pa.Params(fixed_count=0)
    print("[gpu case] warm-start gain: train 256 drops, evaluate 128", flush=True)
    train = [synth.make_drop(synth.CFG2, 2_000_000 + s, 0) for s in range(256)]
    held = [synth.make_drop(synth.CFG2, 3_000_000 + s, 0) for s in range(128)]
    net, info = warm.fit(ctx, train, params, warm.TrainConfig(steps=300, seed=1))
    print(info, flush=True)
    assert info["loss_last"] < 0.5 * info["loss_first"]
    c = warm.compare(ctx, net, held, params)
    print({k: v for k, v in c.items() if k not in ("cold", "warm")}, flush=True)
    ratio = np.array([w.ee / x.ee for w, x in zip(c["warm"], c["cold"])])
    assert c["sweeps_warm"] <= 0.8 * c["sweeps_cold"]
    assert np.median(ratio) >= 0.99
    assert ratio.mean() >= 0.95
    assert c["fallbacks"] <= len(held) // 20
    # the untrained network (same initial weights) does not give the gain
    raw = MLP(ctx, init_params(1))
    c0 = warm.compare(ctx, raw, held[:32], params)
    print("untrained:", {k: v for k, v in c0.items() if k not in ("cold", "warm")}, flush=True)
    ctx.close()
