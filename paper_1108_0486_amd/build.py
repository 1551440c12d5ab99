"""Builds libxg.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1108_0486_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(PKG, "libxg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["xg_kernels.hip", "xg_family.hip", "xg_plan_dev.hip", "xg_static.hip", "xg_util.hip", "xg_api.cpp",
           "xg_serve.cpp", "xg_jump.cpp", "xg_plan.cpp", "xg_tune.cpp"]

# -packed-fp32-ops: no packed FP32 instructions in generated code.
# -ffp-contract=off: every FP32 operation rounds as written (no implicit FMA).
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fvisibility=default",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, out: str | None = None) -> str:
    target = out or LIB_PATH
    tmp = target + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-I", INCLUDE, "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
