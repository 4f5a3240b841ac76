"""Seeded synthetic drops for the PD-NOMA H-CRAN allocator (inputs only).

The generator is shared input infrastructure: it writes channel gains,
user types, streaming traffic and RRH budgets, and holds none of the
allocator's arithmetic.  It is a small C library (``drops.c``) driven through
ctypes; :func:`build` compiles it in place.

Presets follow the workloads of the paper's simulation section (Sec. VIII)
and of the synthetic configurations used for measurement:

* ``cfg1``  M=3 (HPN + 2 LPN), N=8, K=6 (2 streaming), l=2
* ``cfg2``  M=5, N=64, K=32 (8 streaming), l=2
* ``cfg3``  M=17, N=1024, K=256 (64 streaming), l=3
* ``cfg4``  ragged batch: M=1+U{2..16}, N in {64..1024}, K=U{16..256}, K_s=K//4, l=3
* ``paper`` the paper's own channel: chi*d^-3, 42/23 dBm, B_n=31.25 kHz,
  N=32, two LPNs, 125 packets/s of 1024 bits, T=0.2 s
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_libsynth.so")
_lib = None


def build() -> str:
    """Compile drops.c into _libsynth.so (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-fvisibility=hidden",
           "-o", _LIB_PATH, os.path.join(_HERE, "drops.c"), "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


class _Recipe(ctypes.Structure):
    _fields_ = [
        ("cfg_id", ctypes.c_int32), ("M", ctypes.c_int32), ("N", ctypes.c_int32),
        ("K", ctypes.c_int32), ("K_s", ctypes.c_int32), ("path_loss_model", ctypes.c_int32),
        ("cell_radius_m", ctypes.c_double), ("lpn_ring_min_m", ctypes.c_double),
        ("lpn_ring_max_m", ctypes.c_double), ("cluster_radius_m", ctypes.c_double),
        ("cluster_fraction", ctypes.c_double), ("min_dist_m", ctypes.c_double),
        ("shadow_db", ctypes.c_double), ("path_loss_exponent", ctypes.c_double),
        ("bw_hz", ctypes.c_double), ("noise_dbm_hz", ctypes.c_double),
        ("pmax_hpn_dbm", ctypes.c_double), ("pmax_lpn_dbm", ctypes.c_double),
        ("eta_hpn", ctypes.c_double), ("eta_lpn", ctypes.c_double),
        ("rate_bps_lo", ctypes.c_double), ("rate_bps_hi", ctypes.c_double),
        ("delay_lo_s", ctypes.c_double), ("delay_hi_s", ctypes.c_double),
        ("packet_bits", ctypes.c_double),
    ]


class _Out(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "gain", "user_type", "arrival_bps", "delay_s", "pmax_w", "eta", "noise_w",
        "rrh_xy", "user_xy")]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run synth.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_drop.argtypes = [ctypes.POINTER(_Recipe), ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.POINTER(_Out)]
        lib.synth_drop.restype = ctypes.c_int
        lib.synth_philox4x32_10.argtypes = [ctypes.c_void_p] * 3
        lib.synth_philox4x32_10.restype = None
        lib.synth_batch_sizes.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_batch_sizes.restype = None
        _lib = lib
    return _lib


def philox4x32_10(counter, key):
    """Raw Philox4x32-10 block (for known-answer tests)."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    _load().synth_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


@dataclasses.dataclass
class Recipe:
    """Scenario recipe.  Units: metres, Hz, dBm, W, bits, seconds."""
    cfg_id: int
    M: int
    N: int
    K: int
    K_s: int
    l: int
    path_loss_model: int = 0
    cell_radius_m: float = 500.0
    lpn_ring_min_m: float = 100.0
    lpn_ring_max_m: float = 400.0
    cluster_radius_m: float = 50.0
    cluster_fraction: float = 0.5
    min_dist_m: float = 10.0
    shadow_db: float = 8.0
    path_loss_exponent: float = 3.0
    bw_hz: float = 180e3
    noise_dbm_hz: float = -174.0
    pmax_hpn_dbm: float = 46.0
    pmax_lpn_dbm: float = 30.0
    eta_hpn: float = 4.0
    eta_lpn: float = 2.0
    rate_bps_lo: float = 32e3
    rate_bps_hi: float = 256e3
    delay_lo_s: float = 0.020
    delay_hi_s: float = 0.100
    packet_bits: float = 1024.0
    # static power components (W): fibre links and circuits, HPN and per LPN
    p_fiber_hpn: float = 3.0
    p_fiber_lpn: float = 1.0
    p_circuit_hpn: float = 1.0
    p_circuit_lpn: float = 1.0

    def with_sizes(self, M: int, N: int, K: int, K_s: int | None = None) -> "Recipe":
        return dataclasses.replace(self, M=M, N=N, K=K, K_s=(K // 4 if K_s is None else K_s))


@dataclasses.dataclass
class Drop:
    """One synthetic drop (all host arrays)."""
    M: int
    N: int
    K: int
    l: int
    gain: np.ndarray         # float32 [M][N][K]
    user_type: np.ndarray    # uint8 [K]
    arrival_bps: np.ndarray  # float64 [K]
    delay_s: np.ndarray      # float64 [K]
    pmax_w: np.ndarray       # float64 [M]
    eta: np.ndarray          # float64 [M]
    noise_w: float
    bw_hz: float
    packet_bits: float
    p_fiber_hpn: float
    p_fiber_lpn: float
    p_circuit_hpn: float
    p_circuit_lpn: float
    rrh_xy: np.ndarray
    user_xy: np.ndarray
    seed: int = 0
    index: int = 0


def make_drop(rc: Recipe, seed: int = 0, index: int = 0) -> Drop:
    lib = _load()
    M, N, K = rc.M, rc.N, rc.K
    gain = np.empty((M, N, K), dtype=np.float32)
    ut = np.empty(K, dtype=np.uint8)
    arr = np.empty(K, dtype=np.float64)
    dl = np.empty(K, dtype=np.float64)
    pm = np.empty(M, dtype=np.float64)
    eta = np.empty(M, dtype=np.float64)
    nw = np.empty(1, dtype=np.float64)
    rxy = np.empty((M, 2), dtype=np.float64)
    uxy = np.empty((K, 2), dtype=np.float64)
    r = _Recipe(rc.cfg_id, M, N, K, rc.K_s, rc.path_loss_model, rc.cell_radius_m,
                rc.lpn_ring_min_m, rc.lpn_ring_max_m, rc.cluster_radius_m,
                rc.cluster_fraction, rc.min_dist_m, rc.shadow_db, rc.path_loss_exponent,
                rc.bw_hz, rc.noise_dbm_hz, rc.pmax_hpn_dbm, rc.pmax_lpn_dbm, rc.eta_hpn,
                rc.eta_lpn, rc.rate_bps_lo, rc.rate_bps_hi, rc.delay_lo_s, rc.delay_hi_s,
                rc.packet_bits)
    o = _Out(gain.ctypes.data, ut.ctypes.data, arr.ctypes.data, dl.ctypes.data,
             pm.ctypes.data, eta.ctypes.data, nw.ctypes.data, rxy.ctypes.data, uxy.ctypes.data)
    rc_ = lib.synth_drop(ctypes.byref(r), seed, index, ctypes.byref(o))
    if rc_ != 0:
        raise ValueError(f"synth_drop failed with {rc_}")
    return Drop(M, N, K, rc.l, gain, ut, arr, dl, pm, eta, float(nw[0]), rc.bw_hz,
                rc.packet_bits, rc.p_fiber_hpn, rc.p_fiber_lpn, rc.p_circuit_hpn,
                rc.p_circuit_lpn, rxy, uxy, seed, index)


CFG1 = Recipe(cfg_id=1, M=3, N=8, K=6, K_s=2, l=2, rate_bps_lo=64e3, rate_bps_hi=64e3,
              delay_lo_s=0.050, delay_hi_s=0.050)
CFG2 = Recipe(cfg_id=2, M=5, N=64, K=32, K_s=8, l=2)
CFG3 = Recipe(cfg_id=3, M=17, N=1024, K=256, K_s=64, l=3)
CFG4 = Recipe(cfg_id=4, M=0, N=0, K=0, K_s=0, l=3)
# The paper's own simulation channel and traffic (Sec. VIII).
PAPER = Recipe(cfg_id=10, M=3, N=32, K=12, K_s=6, l=2, path_loss_model=1,
               pmax_hpn_dbm=42.0, pmax_lpn_dbm=23.0, bw_hz=31.25e3, shadow_db=0.0,
               rate_bps_lo=128e3, rate_bps_hi=128e3, delay_lo_s=0.2, delay_hi_s=0.2,
               p_fiber_hpn=3.0, p_fiber_lpn=1.0, p_circuit_hpn=3.0, p_circuit_lpn=0.1)

PRESETS = {"cfg1": CFG1, "cfg2": CFG2, "cfg3": CFG3, "paper": PAPER}

# Network architectures compared in the paper's simulation section (Sec. VIII,
# the architecture comparison): the same users and fading, different radio
# access networks on the same sites.  Under the paper's channel
# (chi * d^-psi) a gain does not depend on the tier of the transmitter, so a
# variant changes only which sites transmit, their power budgets and
# efficiencies, and the static power; the solver charges RRH 0 the "hpn"
# static terms and every other RRH the "lpn" ones.
#
# * hcran  the H-CRAN itself: an HPN and M-1 LPN RRHs, PD-NOMA (l users per
#          subcarrier)
# * oma    the same network with one user per subcarrier (l = 1)
# * cran   1-tier C-RAN: LPN RRHs only (an LPN at the HPN's site too)
# * hcn    2-tier HCN: base stations instead of RRHs (no fronthaul), a macro BS
#          at the HPN's site (10 W static) and pico BSs at the LPNs' (6.8 W
#          each), efficiency 4 for all
# * hpn    1-tier HPN: two macro BSs, at the HPN's site and the first LPN's,
#          both with the HPN's power budget, 10 W static and efficiency 4
ARCHITECTURES = ("hcran", "oma", "cran", "hcn", "hpn")
MACRO_STATIC_W = 10.0
PICO_STATIC_W = 6.8
BS_ETA = 4.0


def architecture_drop(arch: str, seed: int = 0, index: int = 0, recipe: Recipe = None) -> Drop:
    """Drop ``index`` of ``seed`` in one of the compared architectures.  All of
    them are cut from the same H-CRAN drop, so they serve the same users over
    the same fading."""
    rc = PAPER if recipe is None else recipe
    if rc.path_loss_model != 1:
        raise ValueError("architectures are defined under the tier-independent channel (chi * d^-psi)")
    if arch not in ARCHITECTURES:
        raise ValueError(f"unknown architecture {arch!r}")
    if arch == "hpn" and rc.M < 2:
        raise ValueError("1-tier HPN needs two sites")
    d = make_drop(rc, seed, index)
    if arch == "oma":
        return dataclasses.replace(d, l=1)
    if arch == "cran":
        return dataclasses.replace(d, pmax_w=np.full(d.M, d.pmax_w[-1]), eta=np.full(d.M, rc.eta_lpn),
                                   p_fiber_hpn=d.p_fiber_lpn, p_circuit_hpn=d.p_circuit_lpn)
    if arch == "hcn":
        return dataclasses.replace(d, eta=np.full(d.M, BS_ETA), p_fiber_hpn=0.0, p_fiber_lpn=0.0,
                                   p_circuit_hpn=MACRO_STATIC_W, p_circuit_lpn=PICO_STATIC_W)
    if arch == "hpn":
        two = slice(0, 2)
        return dataclasses.replace(d, M=2, gain=np.ascontiguousarray(d.gain[two]),
                                   pmax_w=np.full(2, d.pmax_w[0]), eta=np.full(2, BS_ETA),
                                   rrh_xy=d.rrh_xy[two].copy(), p_fiber_hpn=0.0, p_fiber_lpn=0.0,
                                   p_circuit_hpn=MACRO_STATIC_W, p_circuit_lpn=MACRO_STATIC_W)
    return d


CFG4_N_CHOICES = (64, 128, 256, 512, 1024)


def batch_sizes(B: int, seed: int = 0, cfg_id: int = 4, mf=(2, 16), n_choices=CFG4_N_CHOICES,
                k=(16, 256)):
    """Per-drop (M, N, K) of a ragged batch."""
    lib = _load()
    nc = np.asarray(n_choices, dtype=np.int32)
    M = np.empty(B, dtype=np.int32)
    N = np.empty(B, dtype=np.int32)
    K = np.empty(B, dtype=np.int32)
    lib.synth_batch_sizes(seed, cfg_id, B, mf[0], mf[1], nc.ctypes.data, len(nc), k[0], k[1],
                          M.ctypes.data, N.ctypes.data, K.ctypes.data)
    return M, N, K


def make_batch(B: int, seed: int = 0, recipe: Recipe = CFG4, indices=None, threads: int = 1):
    """A ragged batch of drops; drop b uses sizes from batch_sizes and index b.
    With threads > 1 the drops are generated by that many threads (the
    generator releases the interpreter lock; every drop is keyed by its own
    index, so the result does not depend on the thread count)."""
    M, N, K = batch_sizes(B, seed=seed, cfg_id=recipe.cfg_id)
    idx = list(range(B) if indices is None else indices)

    def one(b):
        return make_drop(recipe.with_sizes(int(M[b]), int(N[b]), int(K[b])), seed=seed, index=b)

    if threads <= 1:
        return [one(b) for b in idx]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, idx))
