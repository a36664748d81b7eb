"""Build libfbmc.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfbmc.so")

SOURCES = ["fbmc_kernels.hip", "fbmc_mlp.hip", "fbmc_noalloc.hip", "fbmc_host.cpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # hipcc forms packed FP32 instructions by itself; keep them off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libfbmc.so next to this file."""
    os.makedirs(os.path.join(PKG, "_build"), exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(PKG, "_build", os.path.splitext(src)[0] + ".o")
        cmds.append(["hipcc", *HIPCC_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src),
                     "-I", INCLUDE, "-I", CSRC, "-o", obj])
        objs.append(obj)
    # the sources compile independently: one hipcc process each, at once
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
    failed = [cmd for cmd, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
