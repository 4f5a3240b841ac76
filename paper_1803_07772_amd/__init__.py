"""MI355X energy-efficiency resource allocator for PD-NOMA H-CRANs.

Thin ctypes binding over the C ABI in ``include/alloc.h`` (``_liballoc.so``,
built from ``csrc/alloc.hip`` for gfx950).  Every step of the solve runs in
the HIP kernels; this module only marshals arguments.  There is no CPU
fallback: if the library is missing, importing the solver raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_liballoc.so")

ALLOC_GAIN_ON_DEVICE = 1
ALLOC_OUT_ON_DEVICE = 2
ALLOC_WARM_ON_DEVICE = 4
NOT_CONVERGED = 1
QOS_INFEASIBLE = 2
NEAR_TIE = 4
NONFINITE = 8
SIC_INFEASIBLE = 16
GROUP_TIMEOUT = 32
BUDGET_INFEASIBLE = 64
WARM_FALLBACK = 128

_lib = None


class AllocError(RuntimeError):
    pass


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
                ("stall_sweeps", ctypes.c_int32), ("tol_dinkelbach", ctypes.c_double),
                ("tol_dual", ctypes.c_double), ("step0", ctypes.c_double),
                ("qos_down", ctypes.c_double), ("flags", ctypes.c_uint32), ("max_groups", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("lds_kb", ctypes.c_int32), ("block", ctypes.c_int32),
                ("wave", ctypes.c_int32), ("group_triples", ctypes.c_int32), ("tie_rel", ctypes.c_double),
                ("warm_max_dinkelbach", ctypes.c_int32)]


class _Warm(ctypes.Structure):
    _fields_ = [("p0", ctypes.c_void_p), ("xi0", ctypes.c_void_p), ("zeta0", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("sel", ctypes.c_void_p), ("slot_power", ctypes.c_void_p),
                ("power", ctypes.c_void_p), ("rrh_of_user", ctypes.c_void_p),
                ("xi", ctypes.c_void_p), ("zeta", ctypes.c_void_p),
                ("zeta_sic", ctypes.c_void_p), ("user_rate", ctypes.c_void_p),
                ("ee", ctypes.c_double), ("rate_sum", ctypes.c_double),
                ("power_sum", ctypes.c_double), ("viol_qos", ctypes.c_double),
                ("viol_budget", ctypes.c_double), ("viol_sic", ctypes.c_double),
                ("dinkelbach_iters", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("status_flags", ctypes.c_uint32), ("near_ties", ctypes.c_int32)]


# NumPy mirrors of the C structs (same field order, offsets and size), so
# whole struct arrays are filled column by column.
_PROBLEM_DTYPE = np.dtype({"names": [f for f, _ in _Problem._fields_],
                           "formats": ["<i4"] * 4 + ["<u8"] * 8 + ["<f8"] * 7,
                           "offsets": [getattr(_Problem, f).offset for f, _ in _Problem._fields_],
                           "itemsize": ctypes.sizeof(_Problem)})
_RESULT_DTYPE = np.dtype({"names": [f for f, _ in _Result._fields_],
                          "formats": ["<u8"] * 8 + ["<f8"] * 6 + ["<i4", "<i4", "<u4", "<i4"],
                          "offsets": [getattr(_Result, f).offset for f, _ in _Result._fields_],
                          "itemsize": ctypes.sizeof(_Result)})

EXPORTS = ("alloc_ctx_create", "alloc_ctx_destroy", "alloc_params_default", "alloc_solve",
           "alloc_solve_batch", "alloc_strerror", "alloc_ctx_set_timing", "alloc_ctx_last_kernel_ms",
           "alloc_mlp_create", "alloc_mlp_destroy", "alloc_mlp_set_params", "alloc_mlp_get_params",
           "alloc_mlp_features", "alloc_mlp_forward", "alloc_mlp_grad", "alloc_mlp_train_step",
           "alloc_mlp_adamw", "alloc_mlp_rows", "alloc_mlp_warm", "alloc_solve_mlp",
           "alloc_solve_batch_mlp", "alloc_mlp_last_ms", "alloc_batch_create", "alloc_batch_run",
           "alloc_batch_results", "alloc_batch_last_ms", "alloc_batch_destroy", "alloc_solve_noalloc",
           "alloc_noalloc_max_bytes", "alloc_mlp_save", "alloc_mlp_load")


def load():
    """Load _liballoc.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise AllocError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        lib.alloc_ctx_create.argtypes = [ctypes.c_int, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]
        lib.alloc_ctx_create.restype = ctypes.c_int
        lib.alloc_ctx_destroy.argtypes = [ctypes.c_void_p]
        lib.alloc_ctx_destroy.restype = None
        lib.alloc_params_default.argtypes = [ctypes.POINTER(_Params)]
        lib.alloc_params_default.restype = None
        lib.alloc_solve.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Problem),
                                    ctypes.POINTER(_Params), ctypes.POINTER(_Warm),
                                    ctypes.POINTER(_Result)]
        lib.alloc_solve.restype = ctypes.c_int
        lib.alloc_solve_batch.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(_Problem),
                                          ctypes.POINTER(_Params), ctypes.POINTER(_Warm),
                                          ctypes.POINTER(_Result)]
        lib.alloc_solve_batch.restype = ctypes.c_int
        lib.alloc_strerror.argtypes = [ctypes.c_int]
        lib.alloc_strerror.restype = ctypes.c_char_p
        lib.alloc_ctx_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_int]
        lib.alloc_ctx_set_timing.restype = ctypes.c_int
        lib.alloc_ctx_last_kernel_ms.argtypes = [ctypes.c_void_p]
        lib.alloc_ctx_last_kernel_ms.restype = ctypes.c_double
        lib.alloc_batch_create.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(_Problem),
                                           ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_void_p)]
        lib.alloc_batch_create.restype = ctypes.c_int
        lib.alloc_batch_run.argtypes = [ctypes.c_void_p]
        lib.alloc_batch_run.restype = ctypes.c_int
        lib.alloc_batch_results.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Result)]
        lib.alloc_batch_results.restype = ctypes.c_int
        lib.alloc_batch_last_ms.argtypes = [ctypes.c_void_p]
        lib.alloc_batch_last_ms.restype = ctypes.c_double
        lib.alloc_batch_destroy.argtypes = [ctypes.c_void_p]
        lib.alloc_batch_destroy.restype = None
        lib.alloc_solve_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Problem),
                                            ctypes.POINTER(_Params), ctypes.POINTER(_Result)]
        lib.alloc_solve_noalloc.restype = ctypes.c_int
        lib.alloc_noalloc_max_bytes.argtypes = []
        lib.alloc_noalloc_max_bytes.restype = ctypes.c_size_t
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != 0:
        raise AllocError(f"alloc error {rc}: {load().alloc_strerror(rc).decode()}")


@dataclasses.dataclass
class Params:
    max_dinkelbach: int = 20
    sweeps_per_dinkelbach: int = 200
    refit_period: int = 1
    fixed_count: int = 1
    stall_sweeps: int = 30
    tol_dinkelbach: float = 1e-6
    tol_dual: float = 1e-7
    step0: float = 0.1
    qos_down: float = 0.2
    max_groups: int = 0
    tile: int = 0
    lds_kb: int = 0
    block: int = 0
    wave: int = 0
    group_triples: int = 0
    tie_rel: float = 0.0
    warm_max_dinkelbach: int = 0

    def _c(self, flags: int) -> _Params:
        return _Params(self.max_dinkelbach, self.sweeps_per_dinkelbach, self.refit_period,
                       self.fixed_count, self.stall_sweeps, self.tol_dinkelbach, self.tol_dual,
                       self.step0, self.qos_down, flags, self.max_groups, self.tile, self.lds_kb,
                       self.block, self.wave, self.group_triples, self.tie_rel,
                       self.warm_max_dinkelbach)


def default_params() -> Params:
    p = _Params()
    load().alloc_params_default(ctypes.byref(p))
    return Params(p.max_dinkelbach, p.sweeps_per_dinkelbach, p.refit_period, p.fixed_count,
                  p.stall_sweeps, p.tol_dinkelbach, p.tol_dual, p.step0, p.qos_down, p.max_groups,
                  p.tile, p.lds_kb, p.block, p.wave, p.group_triples, p.tie_rel,
                  p.warm_max_dinkelbach)


@dataclasses.dataclass
class Result:
    sel: np.ndarray
    slot_power: np.ndarray
    rrh_of_user: np.ndarray
    xi: np.ndarray
    zeta: np.ndarray
    zeta_sic: np.ndarray
    user_rate: np.ndarray
    ee: float
    rate_sum: float
    power_sum: float
    dinkelbach_iters: int
    sweeps: int
    status_flags: int
    viol_qos: float = 0.0
    viol_budget: float = 0.0
    viol_sic: float = 0.0
    power: np.ndarray | None = None
    near_ties: int = 0


def _hp(keep, a, dtype):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=dtype)
    keep.append(a)
    return a.ctypes.data


def problem_struct(drop, keep, gain=None, pmask=None, weight=None):
    """(alloc_problem, flags) of a drop; ``gain`` is None (host drop.gain), a
    host array, or a contiguous float32 [M][N][K] GPU tensor."""
    flags = 0
    if gain is not None and hasattr(gain, "data_ptr"):
        if not gain.is_cuda or not gain.is_contiguous() or gain.dtype.itemsize != 4:
            raise ValueError("gain tensor must be contiguous float32 on the GPU")
        if tuple(gain.shape) != (drop.M, drop.N, drop.K):
            raise ValueError(f"gain shape {tuple(gain.shape)} != {(drop.M, drop.N, drop.K)}")
        gptr = gain.data_ptr()
        flags |= ALLOC_GAIN_ON_DEVICE
    else:
        g = drop.gain if gain is None else gain
        if np.shape(g) != (drop.M, drop.N, drop.K):
            raise ValueError("gain shape mismatch")
        gptr = _hp(keep, g, np.float32)
    pb = _Problem(drop.M, drop.N, drop.K, drop.l, gptr, _hp(keep, drop.user_type, np.uint8),
                  _hp(keep, drop.arrival_bps, np.float64), _hp(keep, drop.delay_s, np.float64),
                  _hp(keep, drop.pmax_w, np.float64), _hp(keep, drop.eta, np.float64),
                  _hp(keep, pmask, np.float64), _hp(keep, weight, np.float64),
                  drop.noise_w, drop.bw_hz, drop.packet_bits, drop.p_fiber_hpn,
                  drop.p_fiber_lpn, drop.p_circuit_hpn, drop.p_circuit_lpn)
    return pb, flags


def result_struct(drop, dense_power=False):
    """(alloc_result with host output arrays, the arrays, dense power or None)."""
    M, N, K, L = drop.M, drop.N, drop.K, drop.l
    NP = L * (L - 1) // 2
    out = dict(sel=np.empty((M, N, L), np.int32), slot_power=np.empty((M, N, L)),
               rrh_of_user=np.empty(K, np.int32), xi=np.empty(M), zeta=np.empty(K),
               zeta_sic=np.empty((M, N, NP)), user_rate=np.empty(K))
    dense = np.empty((M, N, K), np.float32) if dense_power else None
    res = _Result(out["sel"].ctypes.data, out["slot_power"].ctypes.data,
                  dense.ctypes.data if dense is not None else None,
                  out["rrh_of_user"].ctypes.data, out["xi"].ctypes.data,
                  out["zeta"].ctypes.data, out["zeta_sic"].ctypes.data if NP else None,
                  out["user_rate"].ctypes.data, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0, 0)
    return res, out, dense


def to_result(res, out, dense) -> "Result":
    return Result(ee=res.ee, rate_sum=res.rate_sum, power_sum=res.power_sum,
                  dinkelbach_iters=res.dinkelbach_iters, sweeps=res.sweeps,
                  status_flags=res.status_flags, viol_qos=res.viol_qos,
                  viol_budget=res.viol_budget, viol_sic=res.viol_sic, power=dense,
                  near_ties=res.near_ties, **out)


class Context:
    """A device context bound to one HIP stream (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream: int | None = None):
        lib = load()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        _check(lib.alloc_ctx_create(device, ctypes.c_void_p(stream), ctypes.byref(h)))
        self._h = h
        self.device = device
        self.timing = False

    def set_timing(self, enable: bool = True):
        """Record HIP events around the solve kernel of each call."""
        _check(load().alloc_ctx_set_timing(self._h, int(enable)))
        self.timing = bool(enable)

    def last_kernel_ms(self) -> float:
        return load().alloc_ctx_last_kernel_ms(self._h)

    def close(self):
        if self._h:
            load().alloc_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve_batch(self, drops, params: Params | None = None, gains=None,
                    dense_power: bool = False, warms=None) -> list:
        """Solve a list of drops in one persistent launch.

        ``gains`` is None (host gains of each drop are copied) or a list of
        contiguous float32 GPU tensors, one [M][N][K] per drop.  ``warms`` is
        None or one dict per drop (keys p0, xi0, zeta0; None for a cold start)
        of host float64 arrays."""
        params = params or Params()
        keep = []
        flags = ALLOC_GAIN_ON_DEVICE if gains is not None else 0
        B = len(drops)
        cwarms = None
        if warms is not None:
            if len(warms) != B:
                raise ValueError("one warm start (or None) per drop")
            cwarms = (_Warm * B)()
            for b, w in enumerate(warms):
                w = w or {}
                cwarms[b] = _Warm(*(_hp(keep, w[k], np.float64) if w.get(k) is not None else None
                                    for k in ("p0", "xi0", "zeta0")))
        probs, results, meta = self._batch_structs(drops, keep, gains, dense_power)
        pc = params._c(flags)
        _check(load().alloc_solve_batch(self._h, B, probs, ctypes.byref(pc), cwarms, results))
        return self._batch_results(results, meta)

    @staticmethod
    def _batch_structs(drops, keep, gains, dense_power):
        """Problem and result structs of a batch.  The per-user and per-RRH
        inputs and every output field live in one host buffer per field,
        drops back to back, and the struct arrays are filled column by
        column (a handful of allocations instead of a dozen per drop); each
        drop's arrays are views into the buffers."""
        B = len(drops)
        if gains is not None and len(gains) != B:
            raise ValueError("one gain tensor per drop")
        M = np.fromiter((d.M for d in drops), np.int64, B)
        N = np.fromiter((d.N for d in drops), np.int64, B)
        K = np.fromiter((d.K for d in drops), np.int64, B)
        L = np.fromiter((d.l for d in drops), np.int64, B)
        NP = L * (L - 1) // 2

        def offsets(n):
            o = np.zeros(B + 1, np.int64)
            np.cumsum(n, out=o[1:])
            return o

        oK, oM, oS, oP = offsets(K), offsets(M), offsets(M * N * L), offsets(M * N * NP)

        def gather(attr, dtype, o):
            buf = np.concatenate([getattr(d, attr) for d in drops], axis=None).astype(dtype, copy=False)
            if buf.size != o[-1]:
                raise ValueError(f"{attr}: sizes do not match the drops")
            buf = np.ascontiguousarray(buf)
            keep.append(buf)
            return buf.ctypes.data

        # gain pointers (device tensors checked as in problem_struct)
        gptr = np.empty(B, np.uint64)
        for b, drop in enumerate(drops):
            shape = (int(M[b]), int(N[b]), int(K[b]))
            g = None if gains is None else gains[b]
            if g is not None:
                if not hasattr(g, "data_ptr"):
                    raise ValueError(f"gain {b} must be a GPU tensor")
                if not g.is_cuda or not g.is_contiguous() or g.dtype.itemsize != 4:
                    raise ValueError("gain tensor must be contiguous float32 on the GPU")
                if tuple(g.shape) != shape:
                    raise ValueError(f"gain shape {tuple(g.shape)} != {shape}")
                gptr[b] = g.data_ptr()
            else:
                if np.shape(drop.gain) != shape:
                    raise ValueError("gain shape mismatch")
                gptr[b] = _hp(keep, drop.gain, np.float32)
        pr = np.zeros(B, _PROBLEM_DTYPE)
        pr["M"], pr["N"], pr["K"], pr["l"] = M, N, K, L
        pr["gain"] = gptr
        pr["user_type"] = gather("user_type", np.uint8, oK) + oK[:-1]
        pr["arrival_bps"] = gather("arrival_bps", np.float64, oK) + 8 * oK[:-1]
        pr["delay_s"] = gather("delay_s", np.float64, oK) + 8 * oK[:-1]
        pr["pmax_w"] = gather("pmax_w", np.float64, oM) + 8 * oM[:-1]
        pr["eta"] = gather("eta", np.float64, oM) + 8 * oM[:-1]
        for f in ("noise_w", "bw_hz", "packet_bits", "p_fiber_hpn", "p_fiber_lpn", "p_circuit_hpn",
                  "p_circuit_lpn"):
            pr[f] = np.fromiter((getattr(d, f) for d in drops), np.float64, B)
        keep.append(pr)
        probs = (_Problem * B).from_buffer(pr)

        out_buf = dict(sel=np.empty(int(oS[-1]), np.int32), slot_power=np.empty(int(oS[-1])),
                       rrh_of_user=np.empty(int(oK[-1]), np.int32), xi=np.empty(int(oM[-1])),
                       zeta=np.empty(int(oK[-1])), zeta_sic=np.empty(max(1, int(oP[-1]))),
                       user_rate=np.empty(int(oK[-1])))
        rs = np.zeros(B, _RESULT_DTYPE)
        for f, o, size in (("sel", oS, 4), ("slot_power", oS, 8), ("rrh_of_user", oK, 4), ("xi", oM, 8),
                           ("zeta", oK, 8), ("zeta_sic", oP, 8), ("user_rate", oK, 8)):
            rs[f] = out_buf[f].ctypes.data + size * o[:-1]
        rs["zeta_sic"][NP == 0] = 0
        dense = [None] * B
        if dense_power:
            oD = offsets(M * N * K)
            dense_buf = np.empty(int(oD[-1]), np.float32)
            rs["power"] = dense_buf.ctypes.data + 4 * oD[:-1]
            dense = [dense_buf[int(oD[b]):int(oD[b + 1])].reshape(int(M[b]), int(N[b]), int(K[b]))
                     for b in range(B)]
        keep.append(rs)
        results = (_Result * B).from_buffer(rs)
        return probs, results, (out_buf, M, N, K, L, NP, oK, oM, oS, oP, list(enumerate(dense)))

    @staticmethod
    def _batch_results(results, meta):
        """Result objects of a batch from _batch_structs' buffers (views)."""
        out_buf, M, N, K, L, NP, oK, oM, oS, oP, outs = meta
        sel, sp, rrh, xi = out_buf["sel"], out_buf["slot_power"], out_buf["rrh_of_user"], out_buf["xi"]
        zeta, zs, ur = out_buf["zeta"], out_buf["zeta_sic"], out_buf["user_rate"]
        M, N, L, NP = M.tolist(), N.tolist(), L.tolist(), NP.tolist()
        oK, oM, oS, oP = oK.tolist(), oM.tolist(), oS.tolist(), oP.tolist()
        rs = []
        for b, dense in outs:
            k0, k1, m0, m1, s0, s1 = oK[b], oK[b + 1], oM[b], oM[b + 1], oS[b], oS[b + 1]
            shape = (M[b], N[b], L[b])
            r = results[b]
            rs.append(Result(sel=sel[s0:s1].reshape(shape), slot_power=sp[s0:s1].reshape(shape),
                             rrh_of_user=rrh[k0:k1], xi=xi[m0:m1], zeta=zeta[k0:k1],
                             zeta_sic=zs[oP[b]:oP[b + 1]].reshape(M[b], N[b], NP[b]),
                             user_rate=ur[k0:k1], ee=r.ee, rate_sum=r.rate_sum,
                             power_sum=r.power_sum, dinkelbach_iters=r.dinkelbach_iters,
                             sweeps=r.sweeps, status_flags=r.status_flags, viol_qos=r.viol_qos,
                             viol_budget=r.viol_budget, viol_sic=r.viol_sic, power=dense,
                             near_ties=int(r.near_ties)))
        return rs

    def solve(self, drop, params: Params | None = None, gain=None, warm=None, pmask=None,
              weight=None, dense_power: bool = False) -> Result:
        """Solve one drop.

        ``gain`` may be a torch tensor on the GPU ([M][N][K] float32, contiguous);
        otherwise ``drop.gain`` (host) is copied by the library.
        ``warm`` is a dict with optional host arrays p0 [M][N][K], xi0 [M], zeta0 [K].
        """
        params = params or Params()
        keep = []
        pb, flags = problem_struct(drop, keep, gain, pmask, weight)
        res, out, dense = result_struct(drop, dense_power)
        wm = None
        if warm is not None:
            wm = _Warm(_hp(keep, warm.get("p0"), np.float64), _hp(keep, warm.get("xi0"), np.float64),
                       _hp(keep, warm.get("zeta0"), np.float64))
        pc = params._c(flags)
        _check(load().alloc_solve(self._h, ctypes.byref(pb), ctypes.byref(pc),
                                  ctypes.byref(wm) if wm is not None else None, ctypes.byref(res)))
        return to_result(res, out, dense)

    def solve_noalloc(self, drop, params: Params | None = None, gain=None, pmask=None, weight=None,
                      dense_power: bool = False) -> Result:
        """Solve one drop (cold start) in the library's fixed device
        workspace: no device memory is allocated (alloc_solve_noalloc)."""
        params = params or Params()
        keep = []
        pb, flags = problem_struct(drop, keep, gain, pmask, weight)
        res, out, dense = result_struct(drop, dense_power)
        pc = params._c(flags)
        _check(load().alloc_solve_noalloc(self._h, ctypes.byref(pb), ctypes.byref(pc), ctypes.byref(res)))
        return to_result(res, out, dense)


def noalloc_max_bytes() -> int:
    """Size of the fixed device workspace of Context.solve_noalloc."""
    return int(load().alloc_noalloc_max_bytes())


class Batch:
    """A resident batch (alloc_batch_*): inputs stay on the device and every
    run replays the captured batched solve."""

    def __init__(self, ctx: Context, drops, params: Params | None = None, gains=None,
                 dense_power: bool = False):
        self.ctx = ctx
        self._keep = []
        self.drops = list(drops)
        self._gains = gains  # device gains must outlive the batch
        flags = ALLOC_GAIN_ON_DEVICE if gains is not None else 0
        probs, results, meta = Context._batch_structs(self.drops, self._keep, gains, dense_power)
        self._results, self._meta = results, meta
        pc = (params or Params())._c(flags)
        h = ctypes.c_void_p()
        _check(load().alloc_batch_create(ctx._h, len(self.drops), probs, ctypes.byref(pc), ctypes.byref(h)))
        self._h = h

    def run(self):
        _check(load().alloc_batch_run(self._h))

    def last_ms(self) -> float:
        return load().alloc_batch_last_ms(self._h)

    def results(self) -> list:
        """Results of the last run (copies: later runs reuse the buffers)."""
        _check(load().alloc_batch_results(self._h, self._results))
        out_buf, *rest, outs = self._meta
        copied = {k: v.copy() for k, v in out_buf.items()}
        outs = [(b, None if dense is None else dense.copy()) for b, dense in outs]
        return Context._batch_results(self._results, (copied, *rest, outs))

    def close(self):
        if getattr(self, "_h", None):
            load().alloc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
