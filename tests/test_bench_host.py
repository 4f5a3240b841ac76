"""Host logic of bench.py (no GPU): the one-GPU guard, the roofline record
and the rule that counter figures are used only for the kernel sources and
batch size they were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_roofline_arithmetic():
    r = bench.roofline("no_such_kernel", 8e9, 2.0)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4000.0)  # 8 GB in 2 ms
    assert r["frac"] == pytest.approx(0.5)
    assert r["traffic"] is None and "valu_issue" not in r


def test_counter_record_needs_matching_sources_and_workload(tmp_path, monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["batch_kernel"]
    wl = rec["workload"]
    if rec["src_sha256"] == bench.solver_source_sha():
        assert bench.traffic_for("batch_kernel", wl) == rec["hbm_bytes_per_launch"]
        assert bench.traffic_for("batch_kernel", wl + "x") is None
        v = bench.valu_issue("batch_kernel", wl, 500.0)
        assert v["frac"] == pytest.approx(rec["valu_wave_insts_per_launch"] / 0.5 / bench.VALU_WAVE_INSTS_PEAK)
    # a record taken on other sources is ignored
    monkeypatch.setattr(bench, "solver_source_sha", lambda: "0" * 64)
    assert bench.traffic_for("batch_kernel", wl) is None
    assert bench.valu_issue("batch_kernel", wl, 500.0) is None


def test_gate_reads_the_stored_subset():
    """The gate's stored oracle results hold the seeded 1% of the ragged
    batch, as the script that writes them selects it."""
    import numpy as np
    from tests.golden import make_cfg4_goldens as mk
    g = np.load(bench.GATE_PATH)
    assert np.array_equal(g["indices"], mk.subset_indices()) and len(g["indices"]) == 41
    for b in g["indices"][:3]:
        assert f"d{b}_sel" in g and f"d{b}_scalars" in g
