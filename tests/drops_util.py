"""Hand-built drops for special-case tests."""
from __future__ import annotations

import numpy as np

import synth


def custom_drop(gain, user_type=None, pmax=None, eta=None, noise=1e-15, l=1, arrival=None,
                delay=None, bw=180e3, packet_bits=1024.0, p_static=(3.0, 1.0, 1.0, 1.0)):
    gain = np.ascontiguousarray(gain, dtype=np.float32)
    M, N, K = gain.shape
    ut = np.zeros(K, np.uint8) if user_type is None else np.asarray(user_type, np.uint8)
    arr = np.zeros(K) if arrival is None else np.asarray(arrival, np.float64)
    dl = np.zeros(K) if delay is None else np.asarray(delay, np.float64)
    pm = np.full(M, 1.0) if pmax is None else np.asarray(pmax, np.float64)
    et = np.full(M, 2.0) if eta is None else np.asarray(eta, np.float64)
    return synth.Drop(M, N, K, l, gain, ut, arr, dl, pm, et, float(noise), float(bw),
                      float(packet_bits), *p_static, np.zeros((M, 2)), np.zeros((K, 2)))


def psi_of(drop):
    import oracle
    return np.array([oracle.min_rate(a, t, drop.packet_bits, drop.bw_hz) if ty else 0.0
                     for a, t, ty in zip(drop.arrival_bps, drop.delay_s, drop.user_type)])
