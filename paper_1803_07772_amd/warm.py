"""Training and evaluation driver of the warm-start network.

The network learns from allocations that the solver itself produces: drops
are solved cold in batches, triples are sampled from each solution (every
selected triple up to a share of the rows, the rest at random), and the
network is trained on those rows with AdamW.  All arithmetic (solves,
features, targets, forward and backward passes, updates) runs in the HIP
kernels; this module only draws indices and moves tensors.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import Context, Params
from .mlp import MLP, Opt, WARM_FALLBACK


@dataclasses.dataclass
class TrainConfig:
    rows_per_drop: int = 2048
    selected_share: float = 0.5   # share of each drop's rows drawn from selected triples
    steps: int = 400
    batch_rows: int = 16384
    lr: float = 2e-3
    weight_decay: float = 1e-4
    seed: int = 0


def solve_cold(ctx: Context, drops, params: Params, gains=None, chunk: int = 512):
    """Cold-start batched solves with dense powers (host results)."""
    out = []
    for i in range(0, len(drops), chunk):
        g = None if gains is None else gains[i:i + chunk]
        out += ctx.solve_batch(drops[i:i + chunk], params, gains=g, dense_power=True)
    return out


def training_rows(net: MLP, drops, results, cfg: TrainConfig, gains=None):
    """(features, targets, weights) GPU tensors of sampled triples."""
    import torch
    rng = np.random.default_rng(cfg.seed)
    feats, targs, wts = [], [], []
    for b, (d, r) in enumerate(zip(drops, results)):
        n3 = d.M * d.N * d.K
        p = r.power.reshape(-1)
        sel = np.flatnonzero(p > 0)
        R = min(cfg.rows_per_drop, n3)
        npos = min(len(sel), int(cfg.selected_share * R))
        pos = rng.choice(sel, npos, replace=False) if npos else np.empty(0, np.int64)
        neg = rng.integers(0, n3, R - npos)
        idx = torch.from_numpy(np.concatenate([pos, neg]).astype(np.int64)).cuda()
        g = None if gains is None else gains[b]
        f, t, w = net.rows(d, torch.from_numpy(r.power).cuda(), torch.from_numpy(r.xi).cuda(),
                           torch.from_numpy(r.zeta).cuda(), idx, gain=g)
        feats.append(f)
        targs.append(t)
        wts.append(w)
    return torch.cat(feats), torch.cat(targs), torch.cat(wts)


def train(net: MLP, feat, target, weight, cfg: TrainConfig):
    """AdamW on random row batches; returns the loss of every step."""
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(cfg.seed)
    R = feat.shape[0]
    opt = Opt(lr=cfg.lr, weight_decay=cfg.weight_decay)
    losses = []
    for s in range(cfg.steps):
        # cosine decay of the step size
        opt.lr = cfg.lr * 0.5 * (1.0 + np.cos(np.pi * s / max(cfg.steps, 1)))
        idx = torch.randint(0, R, (min(cfg.batch_rows, R),), device="cuda", generator=gen)
        losses.append(net.train_step(feat.index_select(0, idx).contiguous(),
                                     target.index_select(0, idx).contiguous(),
                                     weight.index_select(0, idx).contiguous(), opt))
    return losses


def fit(ctx: Context, drops, params: Params, cfg: TrainConfig | None = None, init=None,
        gains=None, chunk: int = 512) -> tuple[MLP, dict]:
    """Solve the training drops cold (``chunk`` drops per batched solve),
    build rows, train a network."""
    from .mlp import init_params
    cfg = cfg or TrainConfig()
    t0 = time.perf_counter()
    results = solve_cold(ctx, drops, params, gains, chunk)
    t1 = time.perf_counter()
    net = MLP(ctx, init_params(cfg.seed) if init is None else init)
    feat, target, weight = training_rows(net, drops, results, cfg, gains)
    t2 = time.perf_counter()
    losses = train(net, feat, target, weight, cfg)
    t3 = time.perf_counter()
    return net, dict(solve_s=t1 - t0, rows_s=t2 - t1, train_s=t3 - t2, rows=int(feat.shape[0]),
                     loss_first=losses[0], loss_last=losses[-1])


def compare(ctx: Context, net: MLP, drops, params: Params, gains=None) -> dict:
    """Cold against warm-started batched solves of the same drops."""
    cold = ctx.solve_batch(drops, params, gains=gains)
    warm = net.solve_batch(drops, params, gains=gains)
    sc = np.array([r.sweeps for r in cold], float)
    sw = np.array([r.sweeps for r in warm], float)
    ec = np.array([r.ee for r in cold])
    ew = np.array([r.ee for r in warm])
    return dict(drops=len(drops), sweeps_cold=float(sc.mean()), sweeps_warm=float(sw.mean()),
                dinkelbach_cold=float(np.mean([r.dinkelbach_iters for r in cold])),
                dinkelbach_warm=float(np.mean([r.dinkelbach_iters for r in warm])),
                ee_ratio_mean=float(np.mean(ew / ec)), ee_ratio_min=float(np.min(ew / ec)),
                fallbacks=int(sum(bool(r.status_flags & WARM_FALLBACK) for r in warm)),
                cold=cold, warm=warm)
