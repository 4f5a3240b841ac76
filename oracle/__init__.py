"""FP64 CPU oracle of the PD-NOMA H-CRAN allocator (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It wraps ``oracle.c`` (plain double-precision C) through ctypes and
shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lib = None

NOT_CONVERGED = 1
QOS_INFEASIBLE = 2
NEAR_TIE = 4
NONFINITE = 8
SIC_INFEASIBLE = 16
BUDGET_INFEASIBLE = 64


def build() -> str:
    """Compile oracle.c into _liboracle.so (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-fvisibility=hidden",
           "-o", _LIB_PATH, os.path.join(_HERE, "oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("N", ctypes.c_int32), ("K", ctypes.c_int32),
                ("l", ctypes.c_int32), ("gain", ctypes.c_void_p), ("user_type", ctypes.c_void_p),
                ("arrival_bps", ctypes.c_void_p), ("delay_s", ctypes.c_void_p),
                ("pmax_w", ctypes.c_void_p), ("eta", ctypes.c_void_p),
                ("pmask_w", ctypes.c_void_p), ("weight", ctypes.c_void_p),
                ("noise_w", ctypes.c_double), ("bw_hz", ctypes.c_double),
                ("packet_bits", ctypes.c_double), ("p_fiber_hpn", ctypes.c_double),
                ("p_fiber_lpn", ctypes.c_double), ("p_circuit_hpn", ctypes.c_double),
                ("p_circuit_lpn", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("max_dinkelbach", ctypes.c_int32), ("sweeps_per_dinkelbach", ctypes.c_int32),
                ("refit_period", ctypes.c_int32), ("fixed_count", ctypes.c_int32),
                ("tol_dinkelbach", ctypes.c_double), ("tol_dual", ctypes.c_double),
                ("step0", ctypes.c_double), ("tie_rel", ctypes.c_double),
                ("stall_sweeps", ctypes.c_int32), ("qos_down", ctypes.c_double)]


class _Warm(ctypes.Structure):
    _fields_ = [("p0", ctypes.c_void_p), ("xi0", ctypes.c_void_p), ("zeta0", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("sel", ctypes.c_void_p), ("slot_power", ctypes.c_void_p),
                ("rrh_of_user", ctypes.c_void_p), ("xi", ctypes.c_void_p),
                ("zeta", ctypes.c_void_p), ("zeta_sic", ctypes.c_void_p),
                ("user_rate", ctypes.c_void_p), ("tie_mn", ctypes.c_void_p),
                ("tie_user", ctypes.c_void_p), ("ee", ctypes.c_double),
                ("rate_sum", ctypes.c_double), ("power_sum", ctypes.c_double),
                ("viol_qos", ctypes.c_double), ("viol_budget", ctypes.c_double),
                ("viol_sic", ctypes.c_double), ("dinkelbach_iters", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("status_flags", ctypes.c_uint32), ("near_ties", ctypes.c_int64),
                ("min_margin", ctypes.c_double), ("first_tie_sweep", ctypes.c_int32),
                ("trace_E", ctypes.c_void_p), ("trace_F", ctypes.c_void_p),
                ("trace_R", ctypes.c_void_p), ("trace_P", ctypes.c_void_p),
                ("trace_sweeps", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run oracle.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        P, R = ctypes.POINTER(_Problem), ctypes.POINTER(_Result)
        lib.orc_solve.argtypes = [P, ctypes.POINTER(_Params), ctypes.POINTER(_Warm), R]
        lib.orc_solve.restype = ctypes.c_int
        lib.orc_state_create.argtypes = [P, ctypes.POINTER(_Params), ctypes.POINTER(_Warm)]
        lib.orc_state_create.restype = ctypes.c_void_p
        lib.orc_state_destroy.argtypes = [ctypes.c_void_p]
        lib.orc_state_set_E.argtypes = [ctypes.c_void_p, ctypes.c_double]
        lib.orc_state_reset_scale.argtypes = [ctypes.c_void_p]
        lib.orc_state_sweep.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
        lib.orc_state_sweep.restype = ctypes.c_double
        lib.orc_state_eval.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4
        lib.orc_state_repair_sic.argtypes = [ctypes.c_void_p]
        lib.orc_state_export.argtypes = [ctypes.c_void_p, R]
        lib.orc_state_get_slots.argtypes = [ctypes.c_void_p] * 6
        lib.orc_state_set_powers.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_state_get_H.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_state_set_multipliers.argtypes = [ctypes.c_void_p] * 4
        lib.orc_min_rate.argtypes = [ctypes.c_double] * 4
        lib.orc_min_rate.restype = ctypes.c_double
        lib.orc_scale_coeffs.argtypes = [ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_sic_margin.argtypes = [ctypes.c_double] * 5
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = ctypes.c_int
        lib.orc_sic_margin.restype = ctypes.c_double
        _lib = lib
    return _lib


@dataclasses.dataclass
class Params:
    max_dinkelbach: int = 20
    sweeps_per_dinkelbach: int = 200
    refit_period: int = 1
    fixed_count: int = 1
    tol_dinkelbach: float = 1e-6
    tol_dual: float = 1e-7
    step0: float = 0.1
    tie_rel: float = 1e-9
    stall_sweeps: int = 30
    qos_down: float = 0.2

    def _c(self) -> _Params:
        return _Params(self.max_dinkelbach, self.sweeps_per_dinkelbach, self.refit_period,
                       self.fixed_count, self.tol_dinkelbach, self.tol_dual, self.step0,
                       self.tie_rel, self.stall_sweeps, self.qos_down)


@dataclasses.dataclass
class Result:
    sel: np.ndarray
    slot_power: np.ndarray
    rrh_of_user: np.ndarray
    xi: np.ndarray
    zeta: np.ndarray
    zeta_sic: np.ndarray
    user_rate: np.ndarray
    tie_mn: np.ndarray
    tie_user: np.ndarray
    ee: float
    rate_sum: float
    power_sum: float
    viol_qos: float
    viol_budget: float
    viol_sic: float
    dinkelbach_iters: int
    sweeps: int
    status_flags: int
    near_ties: int
    min_margin: float
    first_tie_sweep: int
    trace_E: np.ndarray
    trace_F: np.ndarray
    trace_R: np.ndarray
    trace_P: np.ndarray
    trace_sweeps: np.ndarray


class _Keep:
    """Holds the numpy arrays a ctypes struct points into."""

    def __init__(self):
        self.arrs = []

    def ptr(self, a, dtype):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dtype)
        self.arrs.append(a)
        return a.ctypes.data


def _problem(drop, keep: _Keep, pmask=None, weight=None, gain=None) -> _Problem:
    g = drop.gain if gain is None else gain
    return _Problem(drop.M, drop.N, drop.K, drop.l, keep.ptr(g, np.float32),
                    keep.ptr(drop.user_type, np.uint8), keep.ptr(drop.arrival_bps, np.float64),
                    keep.ptr(drop.delay_s, np.float64), keep.ptr(drop.pmax_w, np.float64),
                    keep.ptr(drop.eta, np.float64), keep.ptr(pmask, np.float64),
                    keep.ptr(weight, np.float64), drop.noise_w, drop.bw_hz, drop.packet_bits,
                    drop.p_fiber_hpn, drop.p_fiber_lpn, drop.p_circuit_hpn, drop.p_circuit_lpn)


def _warm(warm, keep: _Keep) -> _Warm | None:
    if warm is None:
        return None
    return _Warm(keep.ptr(warm.get("p0"), np.float64), keep.ptr(warm.get("xi0"), np.float64),
                 keep.ptr(warm.get("zeta0"), np.float64))


def solve(drop, params: Params | None = None, warm=None, pmask=None, weight=None,
          gain=None) -> Result:
    """Full Dinkelbach + SCALE + dual solve of one drop in FP64."""
    lib = _load()
    params = params or Params()
    keep = _Keep()
    M, N, K, L = drop.M, drop.N, drop.K, drop.l
    NP = L * (L - 1) // 2
    out = dict(sel=np.empty((M, N, L), np.int32), slot_power=np.empty((M, N, L)),
               rrh_of_user=np.empty(K, np.int32), xi=np.empty(M), zeta=np.empty(K),
               zeta_sic=np.empty((M, N, NP)), user_rate=np.empty(K),
               tie_mn=np.zeros((M, N), np.int32), tie_user=np.zeros(K, np.int32))
    T = max(params.max_dinkelbach, 1)
    tr = dict(trace_E=np.zeros(T), trace_F=np.zeros(T), trace_R=np.zeros(T),
              trace_P=np.zeros(T), trace_sweeps=np.zeros(T, np.int32))
    res = _Result(*(out[k].ctypes.data for k in ("sel", "slot_power", "rrh_of_user", "xi",
                                                  "zeta", "zeta_sic", "user_rate", "tie_mn",
                                                  "tie_user")),
                  0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0, 0, 0.0, -1,
                  *(tr[k].ctypes.data for k in ("trace_E", "trace_F", "trace_R", "trace_P",
                                                 "trace_sweeps")))
    pb = _problem(drop, keep, pmask, weight, gain)
    wm = _warm(warm, keep)
    rc = lib.orc_solve(ctypes.byref(pb), ctypes.byref(params._c()),
                       ctypes.byref(wm) if wm is not None else None, ctypes.byref(res))
    if rc != 0:
        raise ValueError(f"orc_solve rejected the problem ({rc})")
    n = res.dinkelbach_iters
    return Result(ee=res.ee, rate_sum=res.rate_sum, power_sum=res.power_sum,
                  viol_qos=res.viol_qos, viol_budget=res.viol_budget, viol_sic=res.viol_sic,
                  dinkelbach_iters=n, sweeps=res.sweeps, status_flags=res.status_flags,
                  near_ties=res.near_ties, min_margin=res.min_margin,
                  first_tie_sweep=res.first_tie_sweep,
                  **out, **{k: v[:n] for k, v in tr.items()})


class State:
    """Step-level access to the oracle (for property tests)."""

    def __init__(self, drop, params: Params | None = None, warm=None, pmask=None, weight=None):
        self._lib = _load()
        self._keep = _Keep()
        self.drop = drop
        self.params = params or Params()
        self._pb = _problem(drop, self._keep, pmask, weight)
        self._pc = self.params._c()
        wm = _warm(warm, self._keep)
        self._wm = wm
        self._h = self._lib.orc_state_create(ctypes.byref(self._pb), ctypes.byref(self._pc),
                                             ctypes.byref(wm) if wm is not None else None)
        if not self._h:
            raise ValueError("orc_state_create rejected the problem")

    def close(self):
        if self._h:
            self._lib.orc_state_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_E(self, E: float):
        self._lib.orc_state_set_E(self._h, E)

    def reset_scale(self):
        self._lib.orc_state_reset_scale(self._h)

    def repair_sic(self):
        """Dissolve the pairs that break C14 at the state (as a solve does
        before it returns)."""
        self._lib.orc_state_repair_sic(self._h)

    def sweep(self, v: int, refit: bool) -> float:
        return self._lib.orc_state_sweep(self._h, v, int(refit))

    def evaluate(self):
        R = ctypes.c_double()
        P = ctypes.c_double()
        Rh = ctypes.c_double()
        ur = np.empty(self.drop.K)
        self._lib.orc_state_eval(self._h, ctypes.byref(R), ctypes.byref(P), ctypes.byref(Rh),
                                 ur.ctypes.data)
        return R.value, P.value, Rh.value, ur

    def slots(self):
        """Storage-order slots: (sel [M][N][l], power [M][N][l], xi, zeta, zeta_sic [M][N][l][l])."""
        d = self.drop
        sel = np.empty((d.M, d.N, d.l), np.int32)
        p = np.empty((d.M, d.N, d.l))
        xi = np.empty(d.M)
        zeta = np.empty(d.K)
        zs = np.empty((d.M, d.N, d.l, d.l))
        self._lib.orc_state_get_slots(self._h, sel.ctypes.data, p.ctypes.data, xi.ctypes.data,
                                      zeta.ctypes.data, zs.ctypes.data)
        return sel, p, xi, zeta, zs

    def set_multipliers(self, xi=None, zeta=None, zs=None):
        keep = _Keep()
        self._lib.orc_state_set_multipliers(self._h, keep.ptr(xi, np.float64),
                                            keep.ptr(zeta, np.float64), keep.ptr(zs, np.float64))

    def lagrangian_metric(self):
        """H [M][N][K] of the last sweep."""
        d = self.drop
        H = np.empty((d.M, d.N, d.K))
        self._lib.orc_state_get_H(self._h, H.ctypes.data)
        return H

    def set_powers(self, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        self._lib.orc_state_set_powers(self._h, p.ctypes.data)

    def export(self):
        d = self.drop
        L = d.l
        NP = L * (L - 1) // 2
        out = dict(sel=np.empty((d.M, d.N, L), np.int32), slot_power=np.empty((d.M, d.N, L)),
                   rrh_of_user=np.empty(d.K, np.int32), xi=np.empty(d.M), zeta=np.empty(d.K),
                   zeta_sic=np.empty((d.M, d.N, NP)))
        res = _Result(*(out[k].ctypes.data for k in ("sel", "slot_power", "rrh_of_user", "xi",
                                                      "zeta", "zeta_sic")), None, None, None,
                      0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0, 0, 0.0, -1,
                      None, None, None, None, None)
        self._lib.orc_state_export(self._h, ctypes.byref(res))
        return out


def min_rate(arrival_bps: float, delay_s: float, packet_bits: float, bw_hz: float) -> float:
    return _load().orc_min_rate(arrival_bps, delay_s, packet_bits, bw_hz)


def scale_coeffs(z0: float):
    a = ctypes.c_double()
    b = ctypes.c_double()
    _load().orc_scale_coeffs(z0, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def set_threads(n: int) -> int:
    """Threads of the oracle's loops over subcarriers (n < 1: unchanged);
    returns the previous setting."""
    return _load().orc_set_threads(n)


def sic_margin(g_s, g_w, ici_s, ici_w, sigma) -> float:
    return _load().orc_sic_margin(g_s, g_w, ici_s, ici_w, sigma)
