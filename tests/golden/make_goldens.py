"""Writes the stored oracle results used by the full-size GPU parity test.

Calls only the oracle and the input generator:
    python tests/golden/make_goldens.py
"""
import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def cfg3(seed=0):
    d = synth.make_drop(synth.CFG3, seed, 0)
    r = oracle.solve(d, oracle.Params())  # 200 sweeps per Dinkelbach step, refit every sweep
    np.savez_compressed(
        os.path.join(HERE, f"cfg3_seed{seed}.npz"),
        gain_sha256=np.frombuffer(hashlib.sha256(d.gain.tobytes()).digest(), np.uint8),
        sel=r.sel.astype(np.int16), slot_power=r.slot_power, rrh_of_user=r.rrh_of_user,
        xi=r.xi, zeta=r.zeta, zeta_sic=r.zeta_sic, user_rate=r.user_rate,
        tie_mn=r.tie_mn, tie_user=r.tie_user,
        scalars=np.array([r.ee, r.rate_sum, r.power_sum, r.min_margin]),
        viol=np.array([r.viol_qos, r.viol_budget, r.viol_sic]),
        ints=np.array([r.dinkelbach_iters, r.sweeps, r.status_flags, r.near_ties, r.first_tie_sweep]))
    print("cfg3 seed", seed, "ee", r.ee, "iters", r.dinkelbach_iters, "flags", r.status_flags,
          "ties", r.near_ties, "first tie sweep", r.first_tie_sweep, "min margin", r.min_margin,
          "violations (C13, C12, C14)", r.viol_qos, r.viol_budget, r.viol_sic,
          "flagged (m,n)", int((r.tie_mn > 0).sum()), "flagged users", int((r.tie_user > 0).sum()))


if __name__ == "__main__":
    cfg3(0)
