"""The solver's double-precision logarithms (csrc/logs.h) against the host C
library over arguments spread across the double range: log and log1p within
2 ulp of it, log2 and log2(1 + x) within 3 ulp of references that are
themselves rounded twice (log(x)/log(2)); exact at the special points.  The
harness (tests/logs_probe.hip, built with the package) evaluates them on the
GPU."""
import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_liblogs_probe.so")


def _eval(x, which):
    import torch
    assert torch.cuda.is_available()  # the GPU runtime is torch's before the harness loads
    lib = ctypes.CDLL(LIB)
    lib.logs_probe_eval.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    x = np.ascontiguousarray(x, np.float64)
    y = np.empty_like(x)
    assert lib.logs_probe_eval(x.ctypes.data, y.ctypes.data, x.size, which) == 0
    return y


def _args(positive_only=True):
    rng = np.random.default_rng(7)
    wide = 10.0 ** rng.uniform(-307, 307, 400_000)
    near_one = 1.0 + rng.uniform(-0.3, 0.5, 200_000)
    small = 10.0 ** rng.uniform(-20, 0, 200_000)
    sub = rng.uniform(5e-324, 2.2e-308, 20_000)
    edges = np.array([np.sqrt(0.5), np.nextafter(np.sqrt(0.5), 0), np.sqrt(2.0), 2.0, 0.5, 1e308, 1.7e308,
                      np.nextafter(1.0, 2.0), np.nextafter(1.0, 0.0), 5e-324])
    return np.concatenate([wide, near_one, small, sub, edges])


def _ulps(y, ref):
    return np.abs(y - ref) / np.spacing(np.abs(ref))


def test_log_and_log2_accuracy():
    print("[gpu case] logs: log, log2 on 820k arguments", flush=True)
    x = _args()
    for which, ref_f, bound in ((0, np.log, 2.0), (2, np.log2, 3.0)):
        y, ref = _eval(x, which), ref_f(x)
        ok = ref != 0.0
        err = _ulps(y[ok], ref[ok])
        print(which, "max ulp", err.max(), "mean", err.mean(), flush=True)
        assert err.max() <= bound
        assert np.all(y[~ok] == 0.0)


def test_log1p_and_log2_1p_accuracy():
    print("[gpu case] logs: log1p, log2(1+x) on 820k arguments", flush=True)
    x = np.concatenate([_args(), 10.0 ** np.random.default_rng(8).uniform(-320, -16, 20_000)])
    for which, ref_f, bound in ((1, np.log1p, 2.0), (3, lambda v: np.log1p(v) / np.log(2.0), 3.0)):
        y, ref = _eval(x, which), ref_f(x)
        ok = ref != 0.0
        err = _ulps(y[ok], ref[ok])
        print(which, "max ulp", err.max(), "mean", err.mean(), flush=True)
        assert err.max() <= bound


def test_special_points():
    x = np.array([0.0, 1.0, np.inf, np.nan])
    lg = _eval(x, 0)
    assert lg[0] == -np.inf and lg[1] == 0.0 and lg[2] == np.inf and np.isnan(lg[3])
    l1 = _eval(np.array([0.0, np.inf, np.nan]), 1)
    assert l1[0] == 0.0 and l1[1] == np.inf and np.isnan(l1[2])
