"""Builds libhtree.so (HIP C++ for gfx950) in place, next to this file.

    python -m paper_1406_6158_amd.build

Every source is compiled for gfx950 only, with FP contraction off (the tree
contract writes each fused multiply-add explicitly) and packed-FP32
instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
OUT = PKG / "libhtree.so"
BUILD = ROOT / "_build"
SOURCES = ["build.hip", "force.hip", "integrate.hip", "api.hip", "serve.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-I", str(ROOT / "include"),
]


def _compile(src: str) -> Path:
    obj = BUILD / (Path(src).stem + ".o")
    cmd = [HIPCC, *FLAGS, "-c", str(CSRC / src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s%s" % (src, r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> Path:
    BUILD.mkdir(exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT.with_suffix(".so.tmp%d" % os.getpid())
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


# The host comparison library (cpu/soft_cpu.cpp: the soft interaction loops
# on CPU threads, for the CPU/GPU comparison; never part of the GPU path),
# for any x86-64 host with AVX2 and FMA.
CPU_SRC = PKG / "cpu" / "soft_cpu.cpp"
CPU_OUT = PKG / "libhtree_cpu.so"
CXX = os.environ.get("CXX", "g++")


def build_cpu(verbose: bool = False) -> Path:
    tmp = CPU_OUT.with_suffix(".so.tmp%d" % os.getpid())
    cmd = [CXX, "-O3", "-std=c++17", "-mavx2", "-mfma", "-fPIC", "-shared", "-pthread",
           "-Wall", "-o", str(tmp), str(CPU_SRC)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("g++ failed for %s:\n%s%s" % (CPU_SRC.name, r.stdout, r.stderr))
    os.replace(tmp, CPU_OUT)
    if verbose:
        print("built", CPU_OUT)
    return CPU_OUT


if __name__ == "__main__":
    build(verbose=True)
    build_cpu(verbose=True)
    sys.exit(0)
