"""Build libphiks.so (HIP for gfx950 + host C++) in-tree.

    python paper_2210_07667_amd/build.py

Host planner: g++ -O2.  Device code and C ABI: hipcc --offload-arch=gfx950 -O3 with
packed-FP32 instruction selection disabled.  The library is written next to this
file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libphiks.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed ({' '.join(cmd)}):\n{out}")
    return out


def build(verbose: bool = False, out: str = LIB, build_dir: str = BUILD,
          defines=()) -> str:
    """Compile libphiks.so; `defines` are extra -D flags (tuning variants)."""
    os.makedirs(build_dir, exist_ok=True)
    planner_o = os.path.join(build_dir, "planner.o")
    phiks_o = os.path.join(build_dir, "phiks.o")
    dflags = [f"-D{d}" for d in defines]
    steps = [
        ["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", f"-I{INCLUDE}", "-c",
         os.path.join(CSRC, "planner.cpp"), "-o", planner_o],
        [HIPCC, *HIP_FLAGS, *dflags, f"-I{INCLUDE}", "-c", os.path.join(CSRC, "phiks.hip"),
         "-o", phiks_o],
        [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", planner_o, phiks_o,
         "-lpthread", "-o", out + ".tmp"],
    ]
    for cmd in steps:
        log = _run(cmd)
        if verbose and log.strip():
            print(log)
    shutil.move(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
