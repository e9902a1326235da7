"""Host emulation build of libhtree for CPU tests (no GPU needed).

The library's own sources (csrc/*.hip) are compiled with g++ as C++20
against tests/emu/include/hip/hip_runtime.h, a host stand-in for the HIP
device model, with HTREE_EMU_CHECKS on (every HT_CHECK invariant of the
kernels aborts when broken).  Device pointers are host pointers, so the
ctypes driver below hands numpy buffers straight to the C ABI.  Used only by
tests: the GPU library never includes the stand-in header.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent.parent
CSRC = ROOT / "paper_1406_6158_amd" / "csrc"
EMU_INC = Path(__file__).resolve().parent / "emu" / "include"
OUT = ROOT / "_build" / "libhtree_emu.so"
SOURCES = ["build.hip", "force.hip", "integrate.hip", "api.hip"]

_lib = None


def build(force: bool = False) -> Path:
    srcs = [CSRC / s for s in SOURCES]
    deps = srcs + [CSRC / "htree_dev.h", CSRC / "internal.h", ROOT / "include" / "htree.h",
                   EMU_INC / "hip" / "hip_runtime.h"]
    if not force and OUT.exists() and OUT.stat().st_mtime > max(d.stat().st_mtime for d in deps):
        return OUT
    OUT.parent.mkdir(exist_ok=True)
    tmp = OUT.with_suffix(".so.tmp%d" % os.getpid())
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-DHTREE_EMU_CHECKS", "-Wno-attributes", "-I", str(EMU_INC),
           "-I", str(ROOT / "include"), "-x", "c++", *map(str, srcs), "-o", str(tmp),
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("emulation build failed:\n" + r.stderr[-6000:])
    os.replace(tmp, OUT)
    return OUT


def lib():
    global _lib
    if _lib is None:
        from paper_1406_6158_amd import _abi
        L = C.CDLL(str(build()))
        _p = C.c_void_p
        L.htree_default_params.argtypes = [C.POINTER(_abi.Params)]
        L.htree_workspace_bytes.argtypes = [C.POINTER(_abi.Params), C.c_int64]
        L.htree_workspace_bytes.restype = C.c_size_t
        L.htree_create.argtypes = [C.POINTER(_p), C.POINTER(_abi.Params), C.c_int64, _p,
                                   C.c_size_t, _p]
        L.htree_set_state.argtypes = [_p, _p, _p, _p]
        L.htree_build_tree.argtypes = [_p]
        L.htree_soft_force.argtypes = [_p, _p, _p]
        L.htree_hard_force.argtypes = [_p, _p, _p]
        L.htree_step.argtypes = [_p, C.c_int32]
        L.htree_kick_drift.argtypes = [_p, C.c_double, _p, C.c_double]
        L.htree_refit.argtypes = [_p]
        L.htree_get_state.argtypes = [_p, _p, _p]
        L.htree_sync.argtypes = [_p]
        L.htree_stats.argtypes = [_p, C.POINTER(_abi.Counters)]
        L.htree_group_counts.argtypes = [_p, _p, _p, _p]
        L.htree_group_count.argtypes = [_p]
        L.htree_group_count.restype = C.c_int64
        L.htree_export_groups.argtypes = [_p, _p]
        L.htree_export_keys.argtypes = [_p, _p, _p, _p]
        L.htree_node_count.argtypes = [_p]
        L.htree_node_count.restype = C.c_int64
        L.htree_export_nodes.argtypes = [_p, _p, _p, _p, _p, _p]
        L.htree_export_node_boxes.argtypes = [_p, _p, _p]
        L.htree_last_error.restype = C.c_char_p
        L.htree_destroy.argtypes = [_p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


class EmuTree:
    """One system in the emulated library; arrays are numpy, caller order."""

    def __init__(self, x, v32, m32, **kw):
        from paper_1406_6158_amd import _abi
        L = lib()
        self.n = x.shape[1]
        p = _abi.Params()
        L.htree_default_params(C.byref(p))
        for k, val in kw.items():
            setattr(p, k, val)
        nb = L.htree_workspace_bytes(C.byref(p), self.n)
        assert nb > 0, L.htree_last_error()
        self._ws = np.zeros(nb + 256, np.uint8)
        off = (-self._ws.ctypes.data) % 256
        h = C.c_void_p()
        self._check(L.htree_create(C.byref(h), C.byref(p), self.n,
                                   C.c_void_p(self._ws.ctypes.data + off), nb, None))
        self._h = h
        self._x = np.ascontiguousarray(x, np.float64)
        self._v = None if v32 is None else np.ascontiguousarray(v32, np.float32)
        self._m = np.ascontiguousarray(m32, np.float32)
        self._check(L.htree_set_state(h, _ptr(self._x), _ptr(self._v), _ptr(self._m)))

    def _check(self, code):
        if code != 0:
            raise RuntimeError("htree error %d: %s" % (code, lib().htree_last_error().decode()))

    def build_tree(self):
        self._check(lib().htree_build_tree(self._h))

    def soft_force(self, want_pot=False):
        a = np.zeros((3, self.n), np.float32)
        pot = np.zeros(self.n, np.float32) if want_pot else None
        self._check(lib().htree_soft_force(self._h, _ptr(a), _ptr(pot)))
        return (a, pot) if want_pot else a

    def hard_force(self):
        a = np.zeros((3, self.n), np.float32)
        ngb = np.zeros(self.n, np.int32)
        self._check(lib().htree_hard_force(self._h, _ptr(a), _ptr(ngb)))
        return a, ngb

    def kick_drift(self, dt_kick, dt_drift):
        self._check(lib().htree_kick_drift(self._h, float(dt_kick), None, float(dt_drift)))

    def refit(self):
        self._check(lib().htree_refit(self._h))

    def perm(self):
        """Sorted position -> caller index, of the last build."""
        p = np.zeros(self.n, np.int32)
        self._check(lib().htree_export_keys(self._h, None, _ptr(p), None))
        return p

    def node_ranges(self):
        """(first, count) of every node, in level order."""
        nn = lib().htree_node_count(self._h)
        assert nn >= 0
        first, count = np.zeros(nn, np.int32), np.zeros(nn, np.int32)
        self._check(lib().htree_export_nodes(self._h, None, _ptr(first), _ptr(count), None, None))
        return first, count

    def node_boxes(self):
        nn = lib().htree_node_count(self._h)
        assert nn >= 0
        lo, hi = np.zeros((3, nn)), np.zeros((3, nn))
        self._check(lib().htree_export_node_boxes(self._h, _ptr(lo), _ptr(hi)))
        return lo, hi

    def get_state(self):
        x = np.zeros((3, self.n), np.float64)
        v = np.zeros((3, self.n), np.float32)
        self._check(lib().htree_get_state(self._h, _ptr(x), _ptr(v)))
        return x, v

    def sync(self):
        self._check(lib().htree_sync(self._h))

    def stats(self):
        from paper_1406_6158_amd import _abi
        c = _abi.Counters()
        self._check(lib().htree_stats(self._h, C.byref(c)))
        return c.as_dict()

    def group_starts(self):
        ng = int(lib().htree_group_count(self._h))
        s = np.zeros(ng + 1, np.int32)
        self._check(lib().htree_export_groups(self._h, _ptr(s)))
        return s

    def group_counts(self):
        ng = int(lib().htree_group_count(self._h))
        a = [np.zeros(ng, np.int32) for _ in range(3)]
        self._check(lib().htree_group_counts(self._h, *[_ptr(v) for v in a]))
        return tuple(a)

    def close(self):
        if getattr(self, "_h", None):
            lib().htree_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
