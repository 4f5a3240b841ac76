"""Builds _liballoc.so (and the tests' logarithm harness) for gfx950 with hipcc
(in place, always recompiles)."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off; the compiler emits scalar FP32 instead
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall",
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(_HERE, "csrc", f) for f in ("alloc.hip", "mlp.hip")]
    out = os.path.join(_HERE, "_liballoc.so")
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_logs_probe(verbose: bool = False) -> str:
    """tests/_liblogs_probe.so: the test harness of csrc/logs.h."""
    src = os.path.join(ROOT, "tests", "logs_probe.hip")
    out = os.path.join(ROOT, "tests", "_liblogs_probe.so")
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(_HERE, "csrc"), "-o", tmp, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
