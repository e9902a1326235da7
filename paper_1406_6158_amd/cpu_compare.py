"""The soft interaction loops on host CPU threads, for the CPU/GPU comparison
of section IV.C (the paper runs its force kernels on both kinds of device).

Binds libhtree_cpu.so (built from cpu/soft_cpu.cpp by build.build_cpu).  The
GPU library never calls it: it is a separate host kernel that the benchmark
times beside the GPU soft kernel, and that the tests check against the oracle.
Marshalling only; the arithmetic is in the C++ source.
"""
from __future__ import annotations

import ctypes as C
import os
import time
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "libhtree_cpu.so"
SINKS = 64
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError("%s is not built (paper_1406_6158_amd.build.build_cpu)" % LIB_PATH)
        L = C.CDLL(str(LIB_PATH))
        L.htree_cpu_soft.restype = C.c_int
        L.htree_cpu_soft.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_int64, C.c_float, C.c_float, C.c_float, C.c_void_p,
                                     C.c_int32]
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def soft(sinks, far, near, eps2, R2, invdR, threads=None):
    """Soft accelerations (without G) of groups of 64 sinks.

    sinks [ng][3][64], far [ng][nf][4], near [ng][nn][4] (offsets from each
    group's centre and masses, float32; far or near may be None); returns
    [ng][3][64] float32."""
    sinks = _f32(sinks)
    ng = sinks.shape[0]
    if sinks.shape[1:] != (3, SINKS):
        raise ValueError("sinks must be [ng][3][64]")
    far = None if far is None else _f32(far)
    near = None if near is None else _f32(near)
    nf = 0 if far is None else far.shape[1]
    nn = 0 if near is None else near.shape[1]
    for a in (far, near):
        if a is not None and (a.shape[0] != ng or a.shape[2] != 4):
            raise ValueError("sources must be [ng][count][4]")
    out = np.zeros((ng, 3, SINKS), np.float32)
    threads = threads or os.cpu_count() or 1
    rc = lib().htree_cpu_soft(ng, sinks.ctypes.data, None if far is None else far.ctypes.data, nf,
                              None if near is None else near.ctypes.data, nn, float(eps2),
                              float(R2), float(invdR), out.ctypes.data, int(threads))
    if rc != 0:
        raise ValueError("htree_cpu_soft rejected its arguments")
    return out


def rate(nf, nn, eps2, R2, invdR, groups=256, threads=None, seed=0, repeat=2):
    """Interactions per second of the host loops on `groups` synthetic groups
    with nf far and nn near sources each (sinks within a unit-size group box,
    far sources at 2-10 box sizes, near sources within R2 of the box); the
    best of `repeat` timed calls.  Returns (interactions/s, threads)."""
    rng = np.random.default_rng(seed)
    threads = threads or os.cpu_count() or 1
    sinks = rng.uniform(-0.5, 0.5, (groups, 3, SINKS)).astype(np.float32) * R2
    d = rng.normal(size=(groups, nf, 3))
    d *= (rng.uniform(2.0, 10.0, (groups, nf, 1)) * R2) / np.linalg.norm(d, axis=2, keepdims=True)
    far = np.concatenate([d, np.full((groups, nf, 1), 1e-6)], axis=2).astype(np.float32)
    near = np.concatenate([rng.uniform(-1.5, 1.5, (groups, nn, 3)) * R2,
                           np.full((groups, nn, 1), 1e-6)], axis=2).astype(np.float32)
    best = None
    for _ in range(repeat):
        t0 = time.perf_counter()
        soft(sinks, far, near, eps2, R2, invdR, threads)
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return groups * SINKS * (nf + nn) / best, threads
