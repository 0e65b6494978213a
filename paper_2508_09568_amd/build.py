"""Compile the HIP library libmhdbunch.so for gfx950 (in-tree, next to this file).

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
OBJ = os.path.join(HERE, "csrc", "mhd_bunch.o")
LIB = os.path.join(HERE, "libmhdbunch.so")
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


def torch_lib_dir() -> str:
    import torch
    return os.path.join(os.path.dirname(torch.__file__), "lib")


def build(verbose: bool = False) -> str:
    tl = torch_lib_dir()
    if not os.path.exists(os.path.join(tl, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so in {tl}: a ROCm build of torch is required")
    cmds = [
        [HIPCC, *FLAGS, "-c", SRC, "-o", OBJ],
        ["g++", "-shared", "-o", LIB + ".tmp", OBJ, f"-L{tl}", "-l:libamdhip64.so",
         f"-Wl,-rpath,{tl}", "-Wl,--no-undefined", "-Wl,--no-as-needed"],
    ]
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    os.remove(OBJ)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
