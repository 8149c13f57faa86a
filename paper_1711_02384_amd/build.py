"""Build libc3pt.so (HIP, gfx950) in-tree.

Usage: python paper_1711_02384_amd/build.py  [--debug]
(run as a file: importing the package itself loads the library this builds)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libc3pt.so")
SOURCES = ["c3pt_api.hip", "c3pt_kernels.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, debug: bool = False) -> str:
    flags = [
        "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
        "-O1" if debug else "-O3",
        # packed FP32 instructions are kept out of every kernel of this library
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-Wno-unused-command-line-argument",
    ]
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + flags + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libc3pt.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, debug="--debug" in sys.argv))
