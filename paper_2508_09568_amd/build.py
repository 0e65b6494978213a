"""Compile the HIP library libmhdbunch.so for gfx950 (in-tree, next to this file), and from the
same sources its parity build libmhdbunch_strict.so (no multiply-add contraction, correctly
rounded division and square root: every operation rounded as a plain CPU evaluation of the
same expressions rounds it), which the parity tests use for the comparisons whose bar is
below what contraction changes.

The device code is compiled by hipcc; the shared library is linked against the HIP
runtime that PyTorch loads (its bundled libamdhip64.so), so a process that uses torch
for memory and streams holds exactly one HIP runtime: torch's streams, events and
allocations are then native objects for every launch of this library.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "mhd_bunch.hip")
LIB = os.path.join(HERE, "libmhdbunch.so")
LIB_STRICT = os.path.join(HERE, "libmhdbunch_strict.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: ordinary scalar FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only inside one source expression, never across statements:
    # the same expression then rounds the same wherever it is inlined, so every launch form
    # (tile shapes, solver forms, edge and face lines) gives the same bits by construction
    "-ffp-contract=on",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]
STRICT_FLAGS = [f for f in FLAGS if f != "-ffp-contract=on"] + ["-ffp-contract=off",
                                                                 "-DMHD_STRICT_IEEE"]


def torch_lib_dir() -> str:
    import torch
    return os.path.join(os.path.dirname(torch.__file__), "lib")


def build(verbose: bool = False) -> str:
    """Both libraries, compiled in parallel; returns the path of the product library."""
    tl = torch_lib_dir()
    if not os.path.exists(os.path.join(tl, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so in {tl}: a ROCm build of torch is required")
    jobs = [(LIB, FLAGS), (LIB_STRICT, STRICT_FLAGS)]
    procs = []
    for lib, flags in jobs:
        cmd = [HIPCC, *flags, "-c", SRC, "-o", lib + ".o"]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
    bad = [cmd for cmd, p in procs if p.wait() != 0]
    if bad:
        raise subprocess.CalledProcessError(1, bad[0])
    for lib, _ in jobs:
        cmd = ["g++", "-shared", "-o", lib + ".tmp", lib + ".o", f"-L{tl}", "-l:libamdhip64.so",
               f"-Wl,-rpath,{tl}", "-Wl,--no-undefined", "-Wl,--no-as-needed"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(lib + ".tmp", lib)
        os.remove(lib + ".o")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
