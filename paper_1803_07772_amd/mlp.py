"""Binding of the warm-start network (``include/alloc_mlp.h``).

Argument marshalling only: features, the network's forward and backward
passes, AdamW, pooling and the warm-started solves all run in the HIP kernels
of ``_liballoc.so``.  Data-plane arrays are torch tensors on the GPU.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os

import numpy as np

from . import (AllocError, Context, Params, _Params, _Problem, _Result, _check, load, problem_struct,
               result_struct, to_result)

NIN, HID, NOUT = 4, 256, 3
N_PARAMS = 133635
WARM_FALLBACK = 128
SHAPES = (("W1", (HID, NIN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (NOUT, HID)), ("b4", (NOUT,)))


class _Opt(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("weight_decay", ctypes.c_float)]


@dataclasses.dataclass
class Opt:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    weight_decay: float = 0.01

    def _c(self):
        return _Opt(self.lr, self.beta1, self.beta2, self.eps, self.weight_decay)


_sigs_done = False


def _lib():
    global _sigs_done
    lib = load()
    if not _sigs_done:
        vp, i64, P = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER
        sig = {
            "alloc_mlp_create": ([vp, P(vp)], ctypes.c_int),
            "alloc_mlp_destroy": ([vp], None),
            "alloc_mlp_set_params": ([vp, vp, i64], ctypes.c_int),
            "alloc_mlp_get_params": ([vp, vp, i64], ctypes.c_int),
            "alloc_mlp_features": ([vp, P(_Problem), ctypes.c_uint32, vp], ctypes.c_int),
            "alloc_mlp_forward": ([vp, i64, vp, vp], ctypes.c_int),
            "alloc_mlp_grad": ([vp, i64, vp, vp, vp, vp, P(ctypes.c_double)], ctypes.c_int),
            "alloc_mlp_train_step": ([vp, i64, vp, vp, vp, P(_Opt), P(ctypes.c_double)], ctypes.c_int),
            "alloc_mlp_adamw": ([vp, vp, P(_Opt)], ctypes.c_int),
            "alloc_mlp_rows": ([vp, P(_Problem), ctypes.c_uint32, vp, vp, vp, i64, vp, vp, vp, vp],
                               ctypes.c_int),
            "alloc_mlp_warm": ([vp, P(_Problem), ctypes.c_uint32, vp, vp, vp], ctypes.c_int),
            "alloc_solve_mlp": ([vp, P(_Problem), P(_Params), P(_Result)], ctypes.c_int),
            "alloc_solve_batch_mlp": ([vp, ctypes.c_int32, P(_Problem), P(_Params), P(_Result)],
                                      ctypes.c_int),
            "alloc_mlp_last_ms": ([vp], ctypes.c_double),
            "alloc_mlp_save": ([vp, ctypes.c_char_p], ctypes.c_int),
            "alloc_mlp_load": ([vp, ctypes.c_char_p], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _sigs_done = True
    return lib


def init_params(seed: int = 0) -> np.ndarray:
    """A starting point for training: uniform weights of variance 1/fan_in
    scaled for GELU layers, zero biases (float32, flat parameter order)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SHAPES:
        if name.startswith("W"):
            bound = math.sqrt(6.0 / shape[1])
            parts.append(rng.uniform(-bound, bound, shape).ravel() * (0.5 if name == "W4" else 1.0))
        else:
            parts.append(np.zeros(shape).ravel())
    return np.concatenate(parts).astype(np.float32)


def _dev(t, dtype, shape=None, name="array"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.dtype != dtype:
        raise ValueError(f"{name} must be a contiguous {dtype} GPU tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} shape {tuple(t.shape)} != {tuple(shape)}")
    return t.data_ptr()


class MLP:
    """The warm-start network on one context (and its stream)."""

    def __init__(self, ctx: Context, params: np.ndarray | None = None):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(_lib().alloc_mlp_create(ctx._h, ctypes.byref(h)))
        self._h = h
        if params is not None:
            self.set_params(params)

    def close(self):
        if getattr(self, "_h", None):
            _lib().alloc_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != N_PARAMS:
            raise ValueError(f"{a.size} parameters, expected {N_PARAMS}")
        _check(_lib().alloc_mlp_set_params(self._h, a.ctypes.data, N_PARAMS))

    def get_params(self) -> np.ndarray:
        a = np.empty(N_PARAMS, np.float32)
        _check(_lib().alloc_mlp_get_params(self._h, a.ctypes.data, N_PARAMS))
        return a

    def save(self, path: str):
        """Writes the FP32 master weights (the order alloc_mlp_get_params
        returns) to a safetensors file (alloc_mlp_save); the optimizer's
        moments are not saved."""
        _check(_lib().alloc_mlp_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, ctx: Context, path: str) -> "MLP":
        """A network on ``ctx`` with the weights save() wrote (alloc_mlp_load)."""
        net = cls(ctx)
        try:
            _check(_lib().alloc_mlp_load(net._h, os.fsencode(path)))
        except Exception:
            net.close()
            raise
        return net

    def features(self, drop, gain=None, pmask=None):
        import torch
        keep = []
        pb, flags = problem_struct(drop, keep, gain, pmask)
        out = torch.empty((drop.M * drop.N * drop.K, NIN), dtype=torch.float32, device="cuda")
        _check(_lib().alloc_mlp_features(self._h, ctypes.byref(pb), flags, out.data_ptr()))
        return out

    def forward(self, feat):
        import torch
        R = feat.shape[0]
        _dev(feat, torch.float32, (R, NIN), "feat")
        y = torch.empty((R, NOUT), dtype=torch.float32, device="cuda")
        _check(_lib().alloc_mlp_forward(self._h, R, feat.data_ptr(), y.data_ptr()))
        return y

    def _rows(self, feat, target, weight):
        import torch
        R = feat.shape[0]
        return (R, _dev(feat, torch.float32, (R, NIN), "feat"),
                _dev(target, torch.float32, (R, NOUT), "target"),
                _dev(weight, torch.float32, (R, NOUT), "weight"))

    def grad(self, feat, target, weight):
        """(gradient [N_PARAMS] float32 GPU tensor, mean loss) without an update."""
        import torch
        R, fp, tp, wp = self._rows(feat, target, weight)
        g = torch.empty(N_PARAMS, dtype=torch.float32, device="cuda")
        loss = ctypes.c_double()
        _check(_lib().alloc_mlp_grad(self._h, R, fp, tp, wp, g.data_ptr(), ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, feat, target, weight, opt: Opt | None = None) -> float:
        R, fp, tp, wp = self._rows(feat, target, weight)
        o = (opt or Opt())._c()
        loss = ctypes.c_double()
        _check(_lib().alloc_mlp_train_step(self._h, R, fp, tp, wp, ctypes.byref(o), ctypes.byref(loss)))
        return loss.value

    def adamw(self, grad, opt: Opt | None = None):
        import torch
        _dev(grad, torch.float32, (N_PARAMS,), "grad")
        o = (opt or Opt())._c()
        _check(_lib().alloc_mlp_adamw(self._h, grad.data_ptr(), ctypes.byref(o)))

    def rows(self, drop, power, xi, zeta, idx, gain=None):
        """Training rows of a solved drop at flat triple indices idx (int64 GPU
        tensor); power [M][N][K] float32, xi [M], zeta [K] float64 GPU tensors."""
        import torch
        keep = []
        pb, flags = problem_struct(drop, keep, gain)
        M, N, K = drop.M, drop.N, drop.K
        R = idx.shape[0]
        _dev(idx, torch.int64, (R,), "idx")
        _dev(power, torch.float32, (M, N, K), "power")
        _dev(xi, torch.float64, (M,), "xi")
        _dev(zeta, torch.float64, (K,), "zeta")
        feat = torch.empty((R, NIN), dtype=torch.float32, device="cuda")
        target = torch.empty((R, NOUT), dtype=torch.float32, device="cuda")
        weight = torch.empty((R, NOUT), dtype=torch.float32, device="cuda")
        _check(_lib().alloc_mlp_rows(self._h, ctypes.byref(pb), flags, power.data_ptr(), xi.data_ptr(),
                                     zeta.data_ptr(), R, idx.data_ptr(), feat.data_ptr(),
                                     target.data_ptr(), weight.data_ptr()))
        return feat, target, weight

    def warm(self, drop, gain=None):
        """(p0 [M][N][K], xi0 [M], zeta0 [K]) float64 GPU tensors."""
        import torch
        keep = []
        pb, flags = problem_struct(drop, keep, gain)
        p0 = torch.empty((drop.M, drop.N, drop.K), dtype=torch.float64, device="cuda")
        xi0 = torch.empty(drop.M, dtype=torch.float64, device="cuda")
        zeta0 = torch.empty(drop.K, dtype=torch.float64, device="cuda")
        _check(_lib().alloc_mlp_warm(self._h, ctypes.byref(pb), flags, p0.data_ptr(), xi0.data_ptr(),
                                     zeta0.data_ptr()))
        return p0, xi0, zeta0

    def solve(self, drop, params: Params | None = None, gain=None, dense_power=False):
        """Network inference, then the solve from that warm start (cold-start
        fallback when the warm solve ends non-finite, empty, or infeasible
        for C12 or C13)."""
        keep = []
        pb, flags = problem_struct(drop, keep, gain)
        res, out, dense = result_struct(drop, dense_power)
        pc = (params or Params())._c(flags)
        _check(_lib().alloc_solve_mlp(self._h, ctypes.byref(pb), ctypes.byref(pc), ctypes.byref(res)))
        return to_result(res, out, dense)

    def solve_batch(self, drops, params: Params | None = None, gains=None, dense_power=False):
        keep = []
        flags = 1 if gains is not None else 0
        probs, results, meta = Context._batch_structs(drops, keep, gains, dense_power)
        pc = (params or Params())._c(flags)
        _check(_lib().alloc_solve_batch_mlp(self._h, len(drops), probs, ctypes.byref(pc), results))
        return Context._batch_results(results, meta)

    def last_ms(self) -> float:
        return _lib().alloc_mlp_last_ms(self._h)


__all__ = ["MLP", "Opt", "init_params", "N_PARAMS", "WARM_FALLBACK", "AllocError"]
