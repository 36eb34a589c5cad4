"""Build the HIP library ``libpcf.so`` in-tree for gfx950 with hipcc.

The library is plain C ABI (``include/pcf.h``); this module only runs the
compiler. ``build()`` always recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpcf.so")
SOURCES = ["kernels.hip", "adjoint.hip", "single.hip", "reduce.hip", "abi.hip", "noalloc.hip",
           "plan.cpp"]
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def compile_flags():
    return [
        "--offload-arch=" + ARCH,
        "-O3",
        "-std=c++17",
        "-fPIC",
        # no packed FP32 instructions anywhere in device code; hipcc has no
        # device-only spelling of this -Xclang pair (-Xarch_device refuses
        # it, -mno-packed-fp32-ops does not remove the instructions), so the
        # host pass sees it too and prints that it ignores the feature
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # the tile queue's single-lane ticket atomic stays a plain atomic:
        # the wave-aggregating rewrite would wait for its return right away,
        # in front of the merge work, instead of at the decode after it
        "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
        "-I", os.path.join(ROOT, "include"),
        "-I", CSRC,
        "-Wall",
        "-Wno-unused-function",
    ]


def build(verbose: bool = False) -> str:
    """Compile every source into ``libpcf.so`` (atomic replace)."""
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(build_dir, src + ".o")
        cmd = [hipcc()] + compile_flags() + ["-c", path, "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc()] + [f for f in compile_flags() if f not in ()] + \
                  ["-x", "c++", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
