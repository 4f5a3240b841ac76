"""Writes the stored oracle results of the ragged 4096-drop batch's check
subset: 41 drops (1%) chosen by a seeded permutation, solved by the FP64
oracle in the solver's default converge mode (fixed_count = 0).

Calls only the oracle and the input generator:
    python tests/golden/make_cfg4_goldens.py
Slot powers are stored as float32 (the parity bar on powers is 1e-4
relative); everything else at full precision.
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
B, SEED, SUBSET_SEED, SUBSET = 4096, 0, 4, 41
PATH = os.path.join(HERE, "cfg4_subset.npz")


def subset_indices():
    """The drops of the check subset, in batch order."""
    return np.sort(np.random.default_rng(SUBSET_SEED).permutation(B)[:SUBSET])


def main():
    idx = subset_indices()
    out = {"indices": idx}
    op = oracle.Params(fixed_count=0)
    t0 = time.time()
    for b in idx.tolist():
        d = synth.make_batch(B, seed=SEED, indices=[b])[0]
        r = oracle.solve(d, op)
        p = f"d{b}_"
        out[p + "gain_sha256"] = np.frombuffer(hashlib.sha256(d.gain.tobytes()).digest(), np.uint8)
        out[p + "sel"] = r.sel.astype(np.int16)
        out[p + "slot_power"] = r.slot_power.astype(np.float32)
        out[p + "rrh_of_user"] = r.rrh_of_user.astype(np.int16)
        out[p + "user_rate"] = r.user_rate
        out[p + "xi"] = r.xi
        out[p + "zeta"] = r.zeta
        out[p + "tie_mn"] = np.minimum(r.tie_mn, 255).astype(np.uint8)
        out[p + "tie_user"] = np.minimum(r.tie_user, 255).astype(np.uint8)
        out[p + "scalars"] = np.array([r.ee, r.rate_sum, r.power_sum, r.viol_qos, r.viol_budget,
                                       r.viol_sic])
        out[p + "ints"] = np.array([r.dinkelbach_iters, r.sweeps, r.status_flags, r.near_ties])
        print(f"drop {b} {d.M}x{d.N}x{d.K}: ee {r.ee:.6f} iters {r.dinkelbach_iters} sweeps {r.sweeps} "
              f"flags {r.status_flags} ties {r.near_ties} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(PATH, **out)


if __name__ == "__main__":
    main()
