"""Builds libdsim.so (HIP, gfx950) in the package directory.

    python -m paper_2409_07107_amd.build

Compiles csrc/dsim_api.hip with hipcc for gfx950 only.  Packed FP32
instructions are disabled (-packed-fp32-ops), and so is one backend pass
that miscompiles this source (see `command`).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdsim.so")
SOURCES = [os.path.join(HERE, "csrc", "dsim_api.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("dsim_core.h", "dsim_tree.h", "dsim_ncp.h", "dsim_pipeline.h")] + \
    [os.path.join(ROOT, "include", "dsim.h")]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def command(out: str = LIB, extra=()) -> list:
    # -amdgpu-enable-rewrite-partial-reg-uses=false: with that backend pass
    # on, some inlining outcomes of this source end in a machine-verifier
    # error ("Illegal instruction detected: Operand has incorrect register
    # class" on a compare against the private aperture base) at -O3; the pass
    # only narrows register classes, so turning it off changes no arithmetic.
    return [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-mllvm", "-amdgpu-enable-rewrite-partial-reg-uses=false",
            "-I", os.path.join(ROOT, "include"),
            *extra, *SOURCES, "-o", out]


def build(verbose: bool = True) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
