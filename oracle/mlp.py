"""FP64 reference of the warm-start network (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It shares nothing with the GPU library.  The network is not part of
the paper: it predicts a starting point for the paper's iteration.  The
Dinkelbach method (Sec. III) and the dual loop (Alg. 1) accept any feasible
initial allocation and multipliers, so a better start only changes how many
sweeps are needed.

Network, per triple (m, n, k):

* Features x = [f0, f1, f2, f3]:
  * f0 = (10 log10(Gamma pmask_m / sigma) - 20) / 20, the SNR at the
    spectral mask in dB, centred;
  * f1 = 1 for a streaming user, 0 for an elastic one;
  * f2 = Psi_k, the minimum rate of a streaming user (Sec. II-B), 0 for
    elastic users;
  * f3 = (10 log10(1000 pmax_m) - 40) / 10, the RRH budget in dBm, centred.
* Layers 4 -> 256 -> 256 -> 256 -> 3, GELU after each hidden layer.  GELU is
  the tanh form, 0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).
* Outputs y = [power logit, xi contribution, zeta contribution].

Rounding model of the GPU kernels, emulated here when ``emulate`` is true:

* inputs and weight matrices are rounded to bfloat16 (round to nearest even);
* every product is accumulated exactly (here FP64, there FP32);
* biases stay FP32;
* hidden activations are rounded to bfloat16 before the next layer;
* in the backward pass, every upstream gradient that enters a product
  (dL/dy and dL/dz of each hidden layer) is rounded to bfloat16, and bias
  gradients sum those rounded values.

Loss per row r: BCE-with-logits(y0, t0) + (y1 - t1)^2 + (y2 - t2)^2, each term
times its weight w_rj, averaged over the R rows.

Powers are encoded over P_DECADES decades below the mask: a power p in
[pmask 10^-P_DECADES, pmask] has the code 1 + log10(p/pmask)/P_DECADES in [0, 1].

Warm start from the outputs of every triple of a drop:

* q = sigmoid(y0); p0 = pmask_m 10^(P_DECADES (q - 1)) where q >= Q_MIN, else 0;
* xi0_m = expm1(clip(mean over (n, k) of y1, 0, 30));
* zeta0_k = expm1(clip(mean over (m, n) of y2, 0, 30)) for streaming users,
  0 for elastic ones.

Training targets from a solved drop: t0 = the code of p* clipped to [0, 1]
(0 where p* = 0), t1 = log1p(xi*_m), t2 = log1p(zeta*_k); weights 1, 1 and f1.
"""
from __future__ import annotations

import math

import numpy as np

NIN, HID, NOUT = 4, 256, 3
Q_MIN = 0.1
P_DECADES = 6.0
LOG_CLIP = 30.0
SHAPES = (("W1", (HID, NIN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (NOUT, HID)), ("b4", (NOUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
_GC = math.sqrt(2.0 / math.pi)


def bf16(x) -> np.ndarray:
    """Round to float32, then to bfloat16 by round-to-nearest-even; FP64 out."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def unflatten(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def min_rate(arrival_bps, delay_s, packet_bits, bw_hz):
    """Psi_k (Sec. II-B), the same stable form as the solver oracle."""
    lam = arrival_bps / packet_bits
    x = lam * delay_s
    return arrival_bps / (bw_hz * (1.0 - 1.0 / (x + math.sqrt(1.0 + x * x))))


def features(drop, pmask=None) -> np.ndarray:
    """[M][N][K][4] unrounded features of every triple."""
    M, N, K = drop.M, drop.N, drop.K
    pm = drop.pmax_w / N if pmask is None else np.asarray(pmask, dtype=np.float64)
    g = drop.gain.astype(np.float64)
    X = np.empty((M, N, K, NIN))
    X[..., 0] = (10.0 * np.log10(g * (pm / drop.noise_w)[:, None, None]) - 20.0) / 20.0
    st = drop.user_type.astype(np.float64)
    psi = np.array([min_rate(drop.arrival_bps[k], drop.delay_s[k], drop.packet_bits, drop.bw_hz)
                    if drop.user_type[k] else 0.0 for k in range(K)])
    X[..., 1] = st[None, None, :]
    X[..., 2] = psi[None, None, :]
    X[..., 3] = ((10.0 * np.log10(1000.0 * drop.pmax_w) - 40.0) / 10.0)[:, None, None]
    return X


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(_GC * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    u = _GC * (z + 0.044715 * z ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * _GC * (1.0 + 3.0 * 0.044715 * z * z)


def _r(x, emulate):
    return bf16(x) if emulate else np.asarray(x, dtype=np.float64)


def forward(params: dict, X, emulate: bool = True):
    """y [R][3] and the cache the backward pass needs."""
    X = _r(X, emulate)
    a, cache = X, {"a0": X}
    for i in (1, 2, 3):
        W = _r(params[f"W{i}"], emulate)
        z = a @ W.T + params[f"b{i}"]
        a = _r(gelu(z), emulate)
        cache[f"z{i}"], cache[f"a{i}"] = z, a
    y = a @ _r(params["W4"], emulate).T + params["b4"]
    return y, cache


def loss_terms(y, T, Wt):
    """Per-row loss and dL/dy (before the 1/R average)."""
    y0, t0 = y[:, 0], T[:, 0]
    bce = np.maximum(y0, 0.0) - y0 * t0 + np.log1p(np.exp(-np.abs(y0)))
    sig = 0.5 * (1.0 + np.tanh(0.5 * y0))  # sigmoid without overflow
    l = Wt[:, 0] * bce + Wt[:, 1] * (y[:, 1] - T[:, 1]) ** 2 + Wt[:, 2] * (y[:, 2] - T[:, 2]) ** 2
    dy = np.stack([Wt[:, 0] * (sig - t0), 2.0 * Wt[:, 1] * (y[:, 1] - T[:, 1]),
                   2.0 * Wt[:, 2] * (y[:, 2] - T[:, 2])], axis=1)
    return l, dy


def loss_and_grad(params: dict, X, T, Wt, emulate: bool = True):
    """Mean loss over rows, gradients (same keys as params) and y."""
    R = X.shape[0]
    y, c = forward(params, X, emulate)
    l, dy = loss_terms(y, T, Wt)
    g = {}
    d = _r(dy / R, emulate)
    g["W4"] = d.T @ c["a3"]
    g["b4"] = d.sum(axis=0)
    W = _r(params["W4"], emulate)
    for i in (3, 2, 1):
        da = d @ W
        d = _r(da * gelu_grad(c[f"z{i}"]), emulate)
        g[f"W{i}"] = d.T @ c[f"a{i - 1}"]
        g[f"b{i}"] = d.sum(axis=0)
        W = _r(params[f"W{i}"], emulate)
    return float(l.mean()), g, y


def adamw_step(params: dict, grads: dict, state: dict, lr, beta1=0.9, beta2=0.999, eps=1e-8,
               weight_decay=0.01):
    """One AdamW step (Adam with decoupled weight decay, Loshchilov and Hutter);
    decay applies to the weight matrices only.  Updates params and state."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for name, _ in SHAPES:
        m = state.setdefault("m_" + name, np.zeros_like(params[name]))
        v = state.setdefault("v_" + name, np.zeros_like(params[name]))
        g = grads[name]
        m[...] = beta1 * m + (1.0 - beta1) * g
        v[...] = beta2 * v + (1.0 - beta2) * g * g
        mh = m / (1.0 - beta1 ** t)
        vh = v / (1.0 - beta2 ** t)
        wd = weight_decay if name.startswith("W") else 0.0
        params[name] = params[name] - lr * (mh / (np.sqrt(vh) + eps) + wd * params[name])
    return params


def warm_start(drop, y, pmask=None):
    """(p0 [M][N][K], xi0 [M], zeta0 [K]) from the outputs y [M][N][K][3]."""
    M, N, K = drop.M, drop.N, drop.K
    pm = drop.pmax_w / N if pmask is None else np.asarray(pmask, dtype=np.float64)
    q = 0.5 * (1.0 + np.tanh(0.5 * y[..., 0]))
    p0 = np.where(q >= Q_MIN, pm[:, None, None] * 10.0 ** (P_DECADES * (q - 1.0)), 0.0)
    xi0 = np.expm1(np.clip(y[..., 1].mean(axis=(1, 2)), 0.0, LOG_CLIP))
    z = np.expm1(np.clip(y[..., 2].mean(axis=(0, 1)), 0.0, LOG_CLIP))
    zeta0 = np.where(drop.user_type.astype(bool), z, 0.0)
    return p0, xi0, zeta0


def targets(drop, power, xi, zeta, pmask=None):
    """(T [M][N][K][3], W [M][N][K][3]) from a solved allocation (dense power)."""
    M, N, K = drop.M, drop.N, drop.K
    pm = drop.pmax_w / N if pmask is None else np.asarray(pmask, dtype=np.float64)
    T = np.empty((M, N, K, NOUT))
    pw = np.asarray(power, dtype=np.float64)
    with np.errstate(divide="ignore"):
        code = 1.0 + np.log10(pw / pm[:, None, None]) / P_DECADES
    T[..., 0] = np.where(pw > 0, np.clip(code, 0.0, 1.0), 0.0)
    T[..., 1] = np.log1p(np.asarray(xi, dtype=np.float64))[:, None, None]
    T[..., 2] = np.log1p(np.asarray(zeta, dtype=np.float64))[None, None, :]
    Wt = np.ones((M, N, K, NOUT))
    Wt[..., 2] = drop.user_type.astype(np.float64)[None, None, :]
    return T, Wt
