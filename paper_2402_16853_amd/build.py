"""Build librqa.so (HIP, gfx950) in-tree with hipcc.

Flags that matter for results:
* ``-ffp-contract=off``                  no fused multiply-add in the predicate
* ``-fno-gpu-flush-denormals-to-zero``   IEEE FP32 denormals on the device
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``  no packed FP32 VALU ops
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(REPO, "include")
LIB = os.path.join(HERE, "librqa.so")

SOURCES = ["rqa_tiles.hip", "rqa_api.cpp", "rqa_measures.cpp", "rqa_server.cpp",
           "rqa_static.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("RQA_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-ffp-contract=off", "-fno-fast-math",
    f"--offload-arch={ARCH}",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


CALIB_SRC = "calib.hip"
CALIB_LIB = os.path.join(HERE, "libcalib.so")


def build_calib(verbose: bool = False) -> str:
    """libcalib.so: the VALU-rate calibration kernel used by bench.py --probe-valu."""
    tmp = CALIB_LIB + ".tmp"
    cmd = [HIPCC, "-x", "hip", *COMMON, "-shared", os.path.join(CSRC, CALIB_SRC), "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, CALIB_LIB)
    return CALIB_LIB


def build(verbose: bool = False, save_temps: str | None = None) -> str:
    """Compile every source and link librqa.so (and libcalib.so); always rebuilds."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"]
        cmd = [HIPCC, *lang, *COMMON, "-c", path, "-o", obj]
        if save_temps and src.endswith(".hip"):
            cmd += [f"-save-temps={save_temps}"] if save_temps in ("obj", "cwd") else ["-save-temps"]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True, cwd=objdir)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-Wl,--no-undefined", "-lpthread"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True, cwd=objdir)
    os.replace(tmp, LIB)
    build_calib(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
