"""Build libc3pt.so (HIP, gfx950) in-tree.

Usage: python paper_1711_02384_amd/build.py  [--debug]
(--debug: -O1 and every launch waited for, so a device fault is reported at
the launch that caused it)
(run as a file: importing the package itself loads the library this builds)

Each translation unit is compiled in its own hipcc process (in parallel), then
linked into one shared library next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libc3pt.so")
SOURCES = ["c3pt_api.hip", "c3pt_proj_meson.hip", "c3pt_proj_baryon.hip", "c3pt_proj_insertion.hip",
           "c3pt_combine.hip", "c3pt_phase.hip", "c3pt_batch.hip",
           "c3pt_serve.hip", "c3pt_fac_meson.hip", "c3pt_fac_baryon.hip", "c3pt_fac_insertion.hip",
           "c3pt_gamma.hip", "c3pt_fac_left.hip",
           "c3pt_smear.hip", "c3pt_fs.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, debug: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    flags = [
        "--offload-arch=gfx950", "-std=c++17", "-fPIC",
        "-O1" if debug else "-O3",
        *(["-DC3PT_SYNC_LAUNCHES"] if debug else []),
        # packed FP32 instructions are kept out of every kernel of this library
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-Wno-unused-command-line-argument",
    ]
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc()] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        errs = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write("\n".join(errs) + "\n")
    if failed:
        raise RuntimeError(f"hipcc failed on {failed}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking libc3pt.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, debug="--debug" in sys.argv))
