"""Helpers shared by the GPU tests (test code)."""
from __future__ import annotations


def gpu_params(op, **kw):
    """The solver schedule of oracle parameters ``op`` for the GPU library,
    plus launch-shape fields ``kw``."""
    import paper_1803_07772_amd as pa
    return pa.Params(max_dinkelbach=op.max_dinkelbach,
                     sweeps_per_dinkelbach=op.sweeps_per_dinkelbach,
                     refit_period=op.refit_period, fixed_count=op.fixed_count,
                     stall_sweeps=op.stall_sweeps, tol_dinkelbach=op.tol_dinkelbach,
                     tol_dual=op.tol_dual, step0=op.step0, qos_down=op.qos_down, **kw)
