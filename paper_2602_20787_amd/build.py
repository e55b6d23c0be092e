"""Builds ``libsteps_cyl.so`` (the C-ABI library) in-tree with hipcc for gfx950.

Each HIP source is compiled to its own object (in parallel, under ``_build/``)
and the objects are linked into the shared library; every call recompiles.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libsteps_cyl.so")
SOURCES = sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))
OBJDIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-fvisibility=hidden",
    # packed FP32 VALU instructions stay off: ordinary float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA results in VGPRs: no accumulator-register round trips before the
    # VALU work on them
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
]
# hipcc's host pass warns about the device-only target feature: harmless
_NOISE = ("unknown target feature", "packed-fp32-ops", "warning generated", "warnings generated")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (res.stderr or "").splitlines() if not any(t in ln for t in _NOISE)]
    return res.returncode, msgs


def build(verbose=False, jobs=None):
    """Compile every HIP source and link ``libsteps_cyl.so``; always recompiles."""
    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, os.path.basename(s)[:-4] + ".o") for s in SOURCES]
    cmds = [[HIPCC, *FLAGS, "-c", "-o", o, s] for s, o in zip(SOURCES, objs)]
    if verbose:
        print(" ".join(cmds[0][:-4]) + " -c <src> (x%d)" % len(cmds), flush=True)
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    failed = False
    for s, (rc, msgs) in zip(SOURCES, results):
        if msgs and (rc != 0 or verbose):
            sys.stderr.write("\n".join(msgs) + "\n")
        if rc != 0:
            sys.stderr.write(f"hipcc failed on {os.path.basename(s)} with status {rc}\n")
            failed = True
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    rc, msgs = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    if rc != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError(f"link failed with status {rc}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
