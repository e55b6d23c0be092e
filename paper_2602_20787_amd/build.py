"""Builds ``libsteps_cyl.so`` (the C-ABI library) in-tree with hipcc for gfx950."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(PKG, "libsteps_cyl.so")
SOURCES = sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-fvisibility=hidden",
    # packed FP32 VALU instructions stay off: ordinary float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA results in VGPRs: no accumulator-register round trips before the
    # VALU work on them
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
]


def build(verbose=False):
    """Compile every HIP source into ``libsteps_cyl.so``; always recompiles."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns about the device-only target feature: harmless
    noise = ("unknown target feature", "packed-fp32-ops", "warning generated", "warnings generated")
    msgs = [ln for ln in (res.stderr or "").splitlines() if not any(t in ln for t in noise)]
    if res.returncode != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError(f"hipcc failed with status {res.returncode}")
    if verbose and msgs:
        sys.stderr.write("\n".join(msgs) + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
