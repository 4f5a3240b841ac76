"""Pins of the warm-start network's FP64 reference (oracle/mlp.py).

Each pin ties the reference to something outside itself: torch's own bfloat16
conversion, BCE-with-logits and AdamW (independent library routines), the
erf form of GELU, central finite differences of the loss, and closed forms.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import mlp


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in mlp.SHAPES:
        fan_in = shape[1] if len(shape) == 2 else 1
        p[name] = rng.normal(0.0, scale / math.sqrt(fan_in), shape) if name.startswith("W") \
            else rng.normal(0.0, 0.1, shape)
    return p


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 5000) * 10.0 ** rng.uniform(-30, 30, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, -0.0]])
    x32 = x.astype(np.float32)
    want = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x32), want)
    # ties go to the even mantissa
    assert mlp.bf16(1.0 + 2 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def test_gelu_against_erf_form_and_symmetry():
    z = np.linspace(-8, 8, 4001)
    erf_form = np.array([0.5 * v * (1.0 + math.erf(v / math.sqrt(2.0))) for v in z])
    # the tanh form is a published approximation of z Phi(z); its largest
    # deviation is a few 1e-4
    assert np.max(np.abs(mlp.gelu(z) - erf_form)) < 1e-3
    # z Phi-like forms satisfy gelu(z) - gelu(-z) = z exactly
    assert np.allclose(mlp.gelu(z) - mlp.gelu(-z), z, rtol=0, atol=1e-12)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # derivative against central differences
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(z))) < 1e-8


def test_bce_and_squared_terms_match_torch():
    rng = np.random.default_rng(1)
    R = 200
    y = rng.normal(0, 4, (R, 3))
    T = np.stack([rng.uniform(0, 1, R), rng.normal(0, 1, R), rng.normal(0, 1, R)], axis=1)
    W = rng.uniform(0, 2, (R, 3))
    l, dy = mlp.loss_terms(y, T, W)
    yt = torch.tensor(y, requires_grad=True)
    bce = torch.nn.functional.binary_cross_entropy_with_logits(
        yt[:, 0], torch.tensor(T[:, 0]), weight=torch.tensor(W[:, 0]), reduction="none")
    lt = bce + torch.tensor(W[:, 1]) * (yt[:, 1] - torch.tensor(T[:, 1])) ** 2 + \
        torch.tensor(W[:, 2]) * (yt[:, 2] - torch.tensor(T[:, 2])) ** 2
    lt.sum().backward()
    assert np.allclose(l, lt.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(dy, yt.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_gradients_match_finite_differences():
    """The unrounded backward pass against central differences of the loss."""
    rng = np.random.default_rng(2)
    p = _params(3)
    R = 7
    X = rng.normal(0, 1, (R, 4))
    T = np.stack([rng.uniform(0, 1, R), rng.normal(0, 1, R), rng.normal(0, 1, R)], axis=1)
    Wt = np.ones((R, 3))
    _, g, _ = mlp.loss_and_grad(p, X, T, Wt, emulate=False)
    h = 1e-6
    for name, shape in mlp.SHAPES:
        for idx in [tuple(rng.integers(0, s) for s in shape) for _ in range(6)]:
            pp = {k: v.copy() for k, v in p.items()}
            pp[name][idx] += h
            lp, _, _ = mlp.loss_and_grad(pp, X, T, Wt, emulate=False)
            pp[name][idx] -= 2 * h
            lm, _, _ = mlp.loss_and_grad(pp, X, T, Wt, emulate=False)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g[name][idx])


def test_gradients_match_torch_autograd():
    """The unrounded reference against torch autograd of the same network."""
    rng = np.random.default_rng(4)
    p = _params(5)
    R = 64
    X = rng.normal(0, 1, (R, 4))
    T = np.stack([rng.uniform(0, 1, R), rng.normal(0, 1, R), rng.normal(0, 1, R)], axis=1)
    Wt = rng.uniform(0, 1, (R, 3))
    loss, g, y = mlp.loss_and_grad(p, X, T, Wt, emulate=False)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    a = torch.tensor(X)
    for i in (1, 2, 3):
        a = torch.nn.functional.gelu(a @ tp[f"W{i}"].T + tp[f"b{i}"], approximate="tanh")
    yt = a @ tp["W4"].T + tp["b4"]
    tT, tW = torch.tensor(T), torch.tensor(Wt)
    lt = torch.nn.functional.binary_cross_entropy_with_logits(yt[:, 0], tT[:, 0], weight=tW[:, 0],
                                                              reduction="none")
    lt = lt + tW[:, 1] * (yt[:, 1] - tT[:, 1]) ** 2 + tW[:, 2] * (yt[:, 2] - tT[:, 2]) ** 2
    lt = lt.mean()
    lt.backward()
    assert abs(loss - lt.item()) <= 1e-12 * abs(loss)
    assert np.allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    for k in p:
        assert np.allclose(g[k], tp[k].grad.numpy(), rtol=1e-9, atol=1e-14), k


def test_emulated_rounding_points():
    """With emulation every hidden activation is a bfloat16 value, and the
    emulated output stays within bfloat16 accuracy of the exact one."""
    rng = np.random.default_rng(6)
    p = _params(7)
    X = rng.normal(0, 1, (50, 4))
    y_e, c = mlp.forward(p, X, emulate=True)
    y_x, _ = mlp.forward(p, X, emulate=False)
    for i in (0, 1, 2, 3):
        assert np.array_equal(c[f"a{i}"], mlp.bf16(c[f"a{i}"]))
    assert np.max(np.abs(y_e - y_x)) < 0.05 * np.max(np.abs(y_x))


def test_adamw_matches_torch():
    rng = np.random.default_rng(8)
    p = _params(9)
    tp = {k: torch.tensor(v.copy(), requires_grad=True) for k, v in p.items()}
    decay = [tp[k] for k, _ in mlp.SHAPES if k.startswith("W")]
    nodecay = [tp[k] for k, _ in mlp.SHAPES if not k.startswith("W")]
    opt = torch.optim.AdamW([{"params": decay, "weight_decay": 0.01},
                             {"params": nodecay, "weight_decay": 0.0}],
                            lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    state = {}
    for _ in range(5):
        g = {k: rng.normal(0, 1, v.shape) for k, v in p.items()}
        for k in p:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
        p = mlp.adamw_step(p, g, state, lr=1e-3)
    for k in p:
        assert np.allclose(p[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15), k


def test_adamw_first_step_closed_form():
    """Step 1: m_hat = g and v_hat = g^2, so each weight moves by
    -lr (g/(|g|+eps) + wd theta)."""
    p = _params(10)
    g = {k: np.full_like(v, -0.5) for k, v in p.items()}
    before = {k: v.copy() for k, v in p.items()}
    p = mlp.adamw_step(p, g, {}, lr=0.01, weight_decay=0.1)
    for k in p:
        wd = 0.1 if k.startswith("W") else 0.0
        want = before[k] - 0.01 * (-0.5 / (0.5 + 1e-8) + wd * before[k])
        assert np.allclose(p[k], want, rtol=1e-14, atol=1e-16)


def test_features_closed_form():
    d = synth.make_drop(synth.CFG1, 0, 0)
    X = mlp.features(d)
    pm = d.pmax_w / d.N
    m, n, k = 1, 3, 2
    snr_db = 10 * math.log10(float(d.gain[m, n, k]) * pm[m] / d.noise_w)
    assert X[m, n, k, 0] == pytest.approx((snr_db - 20) / 20, rel=1e-13)
    # 46 dBm HPN and 30 dBm LPN budgets
    assert X[0, 0, 0, 3] == pytest.approx(0.6, abs=1e-9)
    assert X[1, 0, 0, 3] == pytest.approx(-1.0, abs=1e-9)
    # cfg1's streaming users have the worked minimum rate 0.42132 bits/s/Hz
    s = np.flatnonzero(d.user_type)
    assert np.all(X[0, 0, s, 1] == 1.0) and np.allclose(X[0, 0, s, 2], 0.42132, atol=5e-6)
    e = np.flatnonzero(d.user_type == 0)
    assert np.all(X[..., e, 1] == 0.0) and np.all(X[..., e, 2] == 0.0)


def test_warm_start_pooling():
    d = synth.make_drop(synth.CFG1, 0, 0)
    M, N, K = d.M, d.N, d.K
    y = np.zeros((M, N, K, 3))
    y[..., 0] = -10.0  # q ~ 4.5e-5 < Q_MIN: no power
    y[1, 2, 4, 0] = 0.0  # q = 1/2: code 1/2, three decades below the mask
    y[..., 1] = np.log1p(2.0)
    y[0, :, :, 1] = -5.0  # negative mean is clipped to 0
    y[..., 2] = np.log1p(3.0)
    p0, xi0, zeta0 = mlp.warm_start(d, y)
    pm = d.pmax_w / N
    assert p0[1, 2, 4] == pytest.approx(1e-3 * pm[1], rel=1e-13)
    assert np.count_nonzero(p0) == 1
    assert xi0[0] == 0.0 and np.allclose(xi0[1:], 2.0, rtol=1e-13)
    assert np.allclose(zeta0[d.user_type == 1], 3.0, rtol=1e-13)
    assert np.all(zeta0[d.user_type == 0] == 0.0)


def test_targets_from_solution():
    d = synth.make_drop(synth.CFG1, 0, 0)
    pm = d.pmax_w / d.N
    power = np.zeros((d.M, d.N, d.K))
    power[2, 1, 3] = 0.25 * pm[2]
    power[0, 0, 0] = 2.0 * pm[0]  # above the mask: clipped to 1
    power[1, 3, 5] = 1e-9 * pm[1]  # more than six decades below: clipped to 0
    power[1, 4, 5] = 1e-3 * pm[1]  # three decades below: code 1/2
    xi = np.arange(d.M, dtype=np.float64)
    zeta = np.where(d.user_type == 1, 1.5, 0.0)
    T, W = mlp.targets(d, power, xi, zeta)
    assert T[2, 1, 3, 0] == pytest.approx(1.0 + math.log10(0.25) / 6.0, rel=1e-14)
    assert T[0, 0, 0, 0] == 1.0 and T[1, 3, 5, 0] == 0.0
    assert T[1, 4, 5, 0] == pytest.approx(0.5, rel=1e-14)
    assert T[0, 1, 1, 0] == 0.0  # unselected
    assert np.allclose(T[:, 0, 0, 1], np.log1p(xi))
    assert np.all(W[..., 2] == d.user_type[None, None, :])
