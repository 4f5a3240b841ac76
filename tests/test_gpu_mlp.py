"""GPU parity of the warm-start network against its FP64 reference.

The reference (oracle/mlp.py) emulates the kernels' bfloat16 rounding points,
so what remains between the two is FP32-vs-FP64 accumulation (relative
~1e-6) and the bfloat16 roundings it occasionally flips (one bfloat16 ulp,
2^-8 relative, on a small fraction of activations).  Bounds used here:
* outputs: |dy| <= 1e-3 * s + 1e-6 per element, s = sum_h |W4[j,h] a3[h]| + |b4[j]|
  (a flip of every layer-3 activation would move y by at most 2^-8 s);
* gradients: ||dg|| <= 1e-3 ||g|| per tensor (flips are rare and average out);
* AdamW: |dtheta| <= 1e-6 |theta| + 1e-3 lr (one FP32 update).
Weights, features, targets and gradients fed to both sides are generated
here from seeds; nothing the GPU computes is given to the reference.
"""
import dataclasses
import math

import numpy as np
import pytest

import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_1803_07772_amd as pa
    assert torch.cuda.is_available()
    c = pa.Context(0)
    yield c
    c.close()


def _weights(seed, gain=1.5):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in omlp.SHAPES:
        if name.startswith("W"):
            p[name] = rng.normal(0.0, gain / math.sqrt(shape[1]), shape)
        else:
            p[name] = rng.normal(0.0, 0.2, shape)
    flat = omlp.flatten(p).astype(np.float32)
    return flat, omlp.unflatten(flat.astype(np.float64))


def _net(ctx, flat):
    from paper_1803_07772_amd.mlp import MLP
    return MLP(ctx, flat)


def _feat(rng, R):
    X = np.empty((R, 4))
    X[:, 0] = rng.normal(0.5, 1.0, R)
    X[:, 1] = rng.integers(0, 2, R)
    X[:, 2] = X[:, 1] * rng.uniform(0.2, 1.6, R)
    X[:, 3] = rng.choice([0.6, -1.0], R)
    return X.astype(np.float32)


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _output_scale(P, cache):
    W4 = omlp.bf16(P["W4"])
    return np.abs(cache["a3"]) @ np.abs(W4).T + np.abs(P["b4"])


@pytest.mark.parametrize("R", [1, 63, 1000, 4133])
def test_forward_matches_reference(ctx, R):
    print(f"[gpu case] mlp forward R={R}", flush=True)
    flat, P = _weights(0)
    net = _net(ctx, flat)
    X = _feat(np.random.default_rng(R), R)
    y = net.forward(_cuda(X)).cpu().numpy().astype(np.float64)
    yo, cache = omlp.forward(P, X.astype(np.float64), emulate=True)
    s = _output_scale(P, cache)
    err = np.abs(y - yo)
    print("max err / scale", float((err / (s + 1e-30)).max()), flush=True)
    assert np.all(err <= 1e-3 * s + 1e-6)


def test_get_set_params_roundtrip(ctx):
    flat, _ = _weights(1)
    net = _net(ctx, flat)
    assert np.array_equal(net.get_params(), flat)


def test_save_load_roundtrip(ctx, tmp_path):
    """alloc_mlp_save / alloc_mlp_load: the weights come back bit for bit,
    the file is a safetensors file that the safetensors library reads, a
    file that library writes loads, and a file without the right tensor is
    refused with the network unchanged."""
    import paper_1803_07772_amd as pa
    from paper_1803_07772_amd.mlp import MLP
    from safetensors.numpy import load_file, save_file
    print("[gpu case] mlp save/load", flush=True)
    flat, _ = _weights(2)
    net = _net(ctx, flat)
    path = str(tmp_path / "net.safetensors")
    net.save(path)
    back = MLP.load(ctx, path)
    assert np.array_equal(back.get_params(), flat)
    X = _cuda(_feat(np.random.default_rng(9), 300))
    assert np.array_equal(back.forward(X).cpu().numpy(), net.forward(X).cpu().numpy())
    t = load_file(path)
    assert set(t) == {"params"} and np.array_equal(t["params"], flat)
    other, _ = _weights(3)
    ext = str(tmp_path / "ext.safetensors")
    save_file({"params": other}, ext, metadata={"layers": "4-256-256-256-3"})
    b2 = MLP.load(ctx, ext)
    assert np.array_equal(b2.get_params(), other)
    bad = str(tmp_path / "bad.safetensors")
    save_file({"params": flat[:10]}, bad)
    with pytest.raises(pa.AllocError):
        MLP.load(ctx, bad)
    with pytest.raises(pa.AllocError):
        MLP.load(ctx, str(tmp_path / "missing.safetensors"))
    lib = pa.load()
    assert lib.alloc_mlp_load(back._h, bad.encode()) == -2
    assert np.array_equal(back.get_params(), flat)
    for n in (net, back, b2):
        n.close()


def test_features_match_reference(ctx):
    d = synth.make_drop(synth.CFG2, 3, 0)
    print("[gpu case] mlp features cfg2", flush=True)
    flat, _ = _weights(2)
    net = _net(ctx, flat)
    f = net.features(d).cpu().numpy().reshape(d.M, d.N, d.K, 4)
    fo = omlp.features(d)
    assert np.allclose(f[..., 0], fo[..., 0], rtol=1e-6, atol=1e-6)
    assert np.array_equal(f[..., 1], fo[..., 1].astype(np.float32))
    assert np.allclose(f[..., 2], fo[..., 2], rtol=1e-6, atol=0)
    assert np.allclose(f[..., 3], fo[..., 3], rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("R", [300, 5000])
def test_gradients_match_reference(ctx, R):
    print(f"[gpu case] mlp gradients R={R}", flush=True)
    rng = np.random.default_rng(10 + R)
    flat, P = _weights(3)
    net = _net(ctx, flat)
    X = _feat(rng, R)
    T = np.stack([rng.uniform(0, 1, R) * (rng.uniform(size=R) < 0.3), rng.normal(1, 0.5, R),
                  rng.normal(0.5, 0.5, R)], axis=1).astype(np.float32)
    W = np.stack([np.ones(R), np.ones(R), X[:, 1]], axis=1).astype(np.float32)
    g, loss = net.grad(_cuda(X), _cuda(T), _cuda(W))
    g = omlp.unflatten(g.cpu().numpy().astype(np.float64))
    lo, go, _ = omlp.loss_and_grad(P, X.astype(np.float64), T.astype(np.float64), W.astype(np.float64),
                                   emulate=True)
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    for name, _ in omlp.SHAPES:
        rel = np.linalg.norm(g[name] - go[name]) / max(np.linalg.norm(go[name]), 1e-30)
        print(name, "relative gradient error", rel, flush=True)
        assert rel <= 1e-3, name


def test_adamw_matches_reference(ctx):
    print("[gpu case] mlp adamw", flush=True)
    import torch

    from paper_1803_07772_amd.mlp import Opt
    rng = np.random.default_rng(4)
    flat, P = _weights(4)
    net = _net(ctx, flat)
    opt = Opt(lr=2e-3, weight_decay=0.05)
    state = {}
    for _ in range(3):
        gflat = rng.normal(0, 1e-2, flat.size).astype(np.float32)
        net.adamw(torch.from_numpy(gflat).cuda(), opt)
        P = omlp.adamw_step(P, omlp.unflatten(gflat.astype(np.float64)), state, lr=opt.lr,
                            beta1=opt.beta1, beta2=opt.beta2, eps=opt.eps, weight_decay=opt.weight_decay)
    got = net.get_params().astype(np.float64)
    want = omlp.flatten(P)
    assert np.all(np.abs(got - want) <= 1e-6 * np.abs(want) + 1e-3 * opt.lr)


def test_train_step_is_grad_then_adamw(ctx):
    print("[gpu case] mlp train step", flush=True)
    from paper_1803_07772_amd.mlp import Opt
    rng = np.random.default_rng(5)
    flat, _ = _weights(5)
    R = 2048
    X, T, W = _feat(rng, R), rng.uniform(0, 1, (R, 3)).astype(np.float32), np.ones((R, 3), np.float32)
    a, b = _net(ctx, flat), _net(ctx, flat)
    la = a.train_step(_cuda(X), _cuda(T), _cuda(W), Opt())
    g, lb = b.grad(_cuda(X), _cuda(T), _cuda(W))
    b.adamw(g, Opt())
    assert la == lb
    assert np.array_equal(a.get_params(), b.get_params())


def test_training_reduces_loss(ctx):
    """Fitting a smooth function of the features: the loss falls by 10x."""
    print("[gpu case] mlp training", flush=True)
    from paper_1803_07772_amd.mlp import Opt, init_params
    rng = np.random.default_rng(6)
    R = 4096
    X = _feat(rng, R)
    T = np.stack([1 / (1 + np.exp(-2 * X[:, 0])), np.tanh(X[:, 0] + X[:, 3]), X[:, 2] ** 2],
                 axis=1).astype(np.float32)
    W = np.ones((R, 3), np.float32)
    net = _net(ctx, init_params(0))
    Xc, Tc, Wc = _cuda(X), _cuda(T), _cuda(W)
    first = net.train_step(Xc, Tc, Wc, Opt(lr=3e-3))
    bce_floor = float(np.mean(-(T[:, 0] * np.log(T[:, 0]) + (1 - T[:, 0]) * np.log(1 - T[:, 0]))))
    for _ in range(300):
        last = net.train_step(Xc, Tc, Wc, Opt(lr=3e-3))
    print("loss", first, "->", last, "floor", bce_floor, flush=True)
    assert last - bce_floor < 0.1 * (first - bce_floor)


def test_rows_and_warm_start_match_reference(ctx):
    import torch
    d = synth.make_drop(synth.CFG2, 8, 0)
    print("[gpu case] mlp rows + warm start cfg2", flush=True)
    rng = np.random.default_rng(7)
    flat, P = _weights(6)
    net = _net(ctx, flat)
    pm = d.pmax_w / d.N
    power = (np.where(rng.uniform(size=(d.M, d.N, d.K)) < 0.1, 1.0, 0.0)
             * rng.uniform(0, 1.1, (d.M, d.N, d.K)) * pm[:, None, None]).astype(np.float32)
    xi = rng.uniform(0, 4, d.M)
    zeta = np.where(d.user_type == 1, rng.uniform(0, 3, d.K), 0.0)
    idx = rng.choice(d.M * d.N * d.K, 777, replace=False).astype(np.int64)
    f, t, w = net.rows(d, _cuda(power), _cuda(xi), _cuda(zeta), _cuda(idx))
    fo = omlp.features(d).reshape(-1, 4)[idx]
    To, Wo = omlp.targets(d, power, xi, zeta)
    To, Wo = To.reshape(-1, 3)[idx], Wo.reshape(-1, 3)[idx]
    assert np.allclose(f.cpu().numpy(), fo, rtol=1e-6, atol=1e-6)
    assert np.allclose(t.cpu().numpy(), To, rtol=1e-6, atol=1e-7)
    assert np.array_equal(w.cpu().numpy(), Wo.astype(np.float32))

    p0, xi0, zeta0 = (a.cpu().numpy() for a in net.warm(d, gain=torch.from_numpy(d.gain).cuda()))
    yo, cache = omlp.forward(P, omlp.features(d).reshape(-1, 4), emulate=True)
    s = _output_scale(P, cache)
    po, xo, zo = omlp.warm_start(d, yo.reshape(d.M, d.N, d.K, 3))
    # p0: q = sigmoid(y0) moves by at most q(1-q)|dy0|, and p0 by
    # 6 ln(10) p0 dq; entries whose q is that close to the 0.1 threshold may
    # fall either side
    q = 1 / (1 + np.exp(-yo[:, 0]))
    dq = 0.25 * (1e-3 * s[:, 0] + 1e-6)
    sure = np.abs(q - omlp.Q_MIN) > 2 * dq
    pg, po = p0.reshape(-1), po.reshape(-1)
    bound = np.expm1(omlp.P_DECADES * math.log(10.0) * 2 * dq) * po
    assert np.all(np.abs(pg - po)[sure] <= bound[sure] + 1e-300)
    assert np.array_equal(pg[sure] > 0, po[sure] > 0)
    # pooled means move by at most the mean output bound; expm1' = 1 + value
    sx = (1e-3 * s[:, 1] + 1e-6).reshape(d.M, -1).mean(axis=1)
    assert np.all(np.abs(xi0 - xo) <= (1 + xo) * sx * 1.01 + 1e-12)
    sz = (1e-3 * s[:, 2] + 1e-6).reshape(d.M * d.N, d.K).mean(axis=0)
    assert np.all(np.abs(zeta0 - zo) <= (1 + zo) * sz * 1.01 + 1e-12)


def test_solve_mlp_equals_solve_from_its_warm_start(ctx):
    """alloc_solve_mlp = inference + alloc_solve from those arrays (GPU vs GPU),
    and the batched variant agrees with it drop by drop."""
    import paper_1803_07772_amd as pa
    print("[gpu case] solve_mlp consistency", flush=True)
    flat, _ = _weights(7, gain=1.0)
    net = _net(ctx, flat)
    drops = [synth.make_drop(synth.CFG2, 20 + i, i) for i in range(3)]
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=60)
    singles = []
    for d in drops:
        r = net.solve(d, p)
        p0, xi0, zeta0 = (a.cpu().numpy() for a in net.warm(d))
        ref = ctx.solve(d, p, warm=dict(p0=p0, xi0=xi0, zeta0=zeta0))
        if r.status_flags & pa.WARM_FALLBACK:  # the warm solve was judged: the cold one replaced it
            assert needs_fallback(ref)
            ref = ctx.solve(d, p)
        assert r.ee == ref.ee and np.array_equal(r.sel, ref.sel)
        assert np.array_equal(r.slot_power, ref.slot_power)
        singles.append(r)
    batch = net.solve_batch(drops, p)
    for r, b in zip(singles, batch):
        assert abs(r.ee - b.ee) <= 1e-9 * abs(r.ee)
        assert np.array_equal(r.sel, b.sel) and np.array_equal(r.rrh_of_user, b.rrh_of_user)
        assert r.status_flags == b.status_flags


def needs_fallback(r):
    """The warm-started result is replaced by the cold one: non-finite, empty
    (EE <= 0), or infeasible for C12 or C13."""
    import paper_1803_07772_amd as pa
    bad = pa.NONFINITE | pa.QOS_INFEASIBLE | pa.BUDGET_INFEASIBLE
    return bool(r.status_flags & bad) or not r.ee > 0


def test_fallback_on_empty_warm_start(ctx):
    """A network that predicts no power anywhere gives an empty initial
    allocation.  With one Dinkelbach step the warm solve only evaluates it
    (EE 0): the result is the cold solve's, flagged.  With more steps the
    sweeps start from it (an empty allocation breaks C13, so E^1 = 0), the
    solve ends feasible and the warm result stands."""
    import paper_1803_07772_amd as pa
    d = synth.make_drop(synth.CFG1, 0, 0)
    print("[gpu case] warm fallback", flush=True)
    P = {name: np.zeros(shape) for name, shape in omlp.SHAPES}
    P["b4"][0] = -50.0  # q ~ 2e-22 everywhere: p0 = 0
    net = _net(ctx, omlp.flatten(P).astype(np.float32))
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=40, max_dinkelbach=1)
    r = net.solve(d, p)
    cold = ctx.solve(d, p)
    assert r.status_flags == cold.status_flags | pa.WARM_FALLBACK
    assert r.ee == cold.ee and np.array_equal(r.sel, cold.sel)
    pair = [d, synth.make_drop(synth.CFG1, 1, 0)]
    rb = net.solve_batch(pair, p)
    cb = ctx.solve_batch(pair, p)
    for w, c in zip(rb, cb):  # the batched solver reduces in its own fixed order
        assert w.status_flags == c.status_flags | pa.WARM_FALLBACK
        assert w.ee == c.ee and np.array_equal(w.sel, c.sel)
    p4 = dataclasses.replace(p, max_dinkelbach=8)
    r4 = net.solve(d, p4)
    ref = ctx.solve(d, p4, warm=dict(p0=np.zeros((d.M, d.N, d.K)), xi0=None, zeta0=None))
    print(r4.status_flags, r4.ee, ref.ee, flush=True)
    assert not needs_fallback(ref)
    assert not r4.status_flags & pa.WARM_FALLBACK and r4.ee > 0


def test_qos_infeasible_is_a_fallback(ctx):
    """A warm-started solve that ends with a streaming user below its minimum
    rate (here unreachable) is replaced by the cold solve, flagged; the cold
    result keeps its own flags."""
    import paper_1803_07772_amd as pa
    d = synth.make_drop(synth.CFG1, 0, 0)
    d = dataclasses.replace(d, arrival_bps=d.arrival_bps.copy())
    s = int(np.flatnonzero(d.user_type)[0])
    d.arrival_bps[s] = 5e8  # ~2800 bits/s/Hz: unreachable
    print("[gpu case] qos-infeasible warm solve", flush=True)
    flat, _ = _weights(8, gain=1.0)
    net = _net(ctx, flat)
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=40, max_dinkelbach=4)
    r = net.solve(d, p)
    cold = ctx.solve(d, p)
    assert cold.status_flags & pa.QOS_INFEASIBLE
    assert r.status_flags == cold.status_flags | pa.WARM_FALLBACK
    assert r.ee == cold.ee and np.array_equal(r.sel, cold.sel)


def test_warm_attempt_capped(ctx):
    """alloc_params.warm_max_dinkelbach: a warm attempt that meets the
    stopping test within the cap is the uncapped warm result, bit for bit; one
    that needs more Dinkelbach steps than the cap is replaced by the cold
    solve (which keeps the full max_dinkelbach), flagged."""
    import paper_1803_07772_amd as pa
    d = synth.make_drop(synth.CFG1, 2, 0)
    print("[gpu case] capped warm attempt", flush=True)
    flat, _ = _weights(8, gain=1.0)
    net = _net(ctx, flat)
    p = pa.Params(fixed_count=0, sweeps_per_dinkelbach=200, max_dinkelbach=20)
    free = net.solve(d, p)
    assert not free.status_flags & pa.WARM_FALLBACK
    D = free.dinkelbach_iters
    assert 2 <= D < 20
    same = net.solve(d, dataclasses.replace(p, warm_max_dinkelbach=D))
    assert same.ee == free.ee and np.array_equal(same.sel, free.sel) and same.status_flags == free.status_flags
    cut = net.solve(d, dataclasses.replace(p, warm_max_dinkelbach=D - 1))
    cold = ctx.solve(d, p)
    assert cut.status_flags == cold.status_flags | pa.WARM_FALLBACK
    assert cut.ee == cold.ee and np.array_equal(cut.sel, cold.sel)
    rb = net.solve_batch([d], dataclasses.replace(p, warm_max_dinkelbach=D - 1))[0]
    assert rb.status_flags & pa.WARM_FALLBACK or (rb.dinkelbach_iters <= D - 1 and
                                                  not rb.status_flags & pa.NOT_CONVERGED)
    net.close()
