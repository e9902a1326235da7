"""FP64 CPU oracle for the hybrid hard/soft tree force path (ctypes shim).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does and shares
no code with it.  The arithmetic lives in ``htree_oracle.c`` (plain C, FP64,
built with -ffp-contract=off); this module only marshals numpy arrays.

Every wrapper takes positions as float64 arrays of shape (3, n) and masses as
float64 (n,), in the caller's particle order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "htree_oracle.c"
_LIB = _HERE / "liboracle.so"

_i64 = C.c_int64
_i32 = C.c_int32
_f64 = C.c_double
_p = C.c_void_p


def build(force: bool = False) -> Path:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-std=c11", "-o", str(tmp), str(_SRC), "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(str(build()))
        L.orc_version.restype = C.c_int
        L.orc_threads.restype = C.c_int
        L.orc_K.restype = _f64
        L.orc_K.argtypes = [_f64]
        L.orc_interleave.restype = C.c_uint64
        L.orc_interleave.argtypes = [C.c_uint32] * 3
        L.orc_direct.argtypes = [_i64, _p, _p, _f64, _f64, _i64, _p, _p, _p]
        L.orc_split_direct.argtypes = [_i64, _p, _p, _f64, _f64, _f64, _f64, _i64, _p, _p, _p, _p]
        L.orc_energy.argtypes = [_i64, _p, _p, _p, _f64, _f64, _p, _p]
        L.orc_tree_build.restype = _p
        L.orc_tree_build.argtypes = [_i64, _p, _p, _i32, _f64]
        L.orc_tree_free.argtypes = [_p]
        L.orc_tree_nnodes.restype = _i64
        L.orc_tree_nnodes.argtypes = [_p]
        L.orc_tree_frame.argtypes = [_p, _p, _p]
        L.orc_tree_sorted.argtypes = [_p, _p, _p, _p]
        L.orc_tree_nodes.argtypes = [_p] * 11
        L.orc_tree_set_mac.argtypes = [_p, _f64, _f64, _i32]
        L.orc_tree_node_mac.argtypes = [_p, _p, _p]
        L.orc_tree_groups.restype = _i64
        L.orc_tree_groups.argtypes = [_p, _i32, _i32]
        L.orc_tree_group_starts.argtypes = [_p, _p]
        L.orc_walk_counts.argtypes = [_p, _f64, _i32, _p, _p, _p]
        L.orc_walk_group.argtypes = [_p, _i64, _f64, _i32, _i64, _p, _p, _p, _p]
        L.orc_soft.restype = _i64
        L.orc_soft.argtypes = [_p, _f64, _f64, _f64, _f64, _i32, _i64, _p, _p, _p]
        L.orc_step.argtypes = [_i64, _p, _p, _p, _f64, _f64, _f64, _f64, _f64, _i32, _i32,
                               _i32, _i32, _f64, _i32, _i32]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def threads() -> int:
    return lib().orc_threads()


def K(Y: float) -> float:
    """Changeover function of section II.C, eq. (10)."""
    return lib().orc_K(float(Y))


def interleave(qx: int, qy: int, qz: int) -> int:
    return int(lib().orc_interleave(qx, qy, qz))


def direct(x, m, G=1.0, eps=0.0, sinks=None, potential=False):
    """Direct-sum acceleration (3, ns) and optional potential (ns,)."""
    x = _f64c(x)
    m = _f64c(m)
    n = x.shape[1]
    s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
    ns = n if s is None else s.size
    acc = np.zeros((3, ns))
    pot = np.zeros(ns) if potential else None
    lib().orc_direct(n, _ptr(x), _ptr(m), G, eps, ns, _ptr(s), _ptr(acc), _ptr(pot))
    return (acc, pot) if potential else acc


def split_direct(x, m, G, eps, R1, R2, sinks=None, soft=True):
    """Direct hard/soft split: returns (a_hard, a_soft or None, ngb)."""
    x = _f64c(x)
    m = _f64c(m)
    n = x.shape[1]
    s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
    ns = n if s is None else s.size
    ah = np.zeros((3, ns))
    aso = np.zeros((3, ns)) if soft else None
    ngb = np.zeros(ns, dtype=np.int64)
    lib().orc_split_direct(n, _ptr(x), _ptr(m), G, eps, R1, R2, ns, _ptr(s),
                           _ptr(ah), _ptr(aso), _ptr(ngb))
    return ah, aso, ngb


def energy(x, v, m, G=1.0, eps=0.0):
    """(kinetic, potential) energy, potential by direct summation."""
    x = _f64c(x)
    m = _f64c(m)
    v = None if v is None else _f64c(v)
    kin = C.c_double()
    pot = C.c_double()
    lib().orc_energy(x.shape[1], _ptr(x), _ptr(v), _ptr(m), G, eps,
                     C.byref(kin), C.byref(pot))
    return kin.value, pot.value


class Tree:
    """The oracle's octree over a particle set (built on construction)."""

    def __init__(self, x, m, n_crit=16, theta=0.5, group=64, chunk=16):
        self.x = _f64c(x)
        self.m = _f64c(m)
        self.n = self.x.shape[1]
        self.theta = float(theta)
        self.n_crit = int(n_crit)
        self._h = lib().orc_tree_build(self.n, _ptr(self.x), _ptr(self.m), self.n_crit,
                                       self.theta)
        if not self._h:
            raise ValueError("oracle tree build rejected its arguments")
        self.g = int(group)
        self.chunk = int(chunk)
        self.ngroups = int(lib().orc_tree_groups(self._h, self.g, self.chunk))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_tree_free(h)
            self._h = None

    @property
    def nnodes(self) -> int:
        return int(lib().orc_tree_nnodes(self._h))

    def frame(self):
        lo = np.zeros(3)
        side = C.c_double()
        lib().orc_tree_frame(self._h, _ptr(lo), C.byref(side))
        return lo, side.value

    def sorted(self):
        """(perm, keys, u): sorted position -> caller index, keys, build-frame positions."""
        perm = np.zeros(self.n, dtype=np.int64)
        key = np.zeros(self.n, dtype=np.uint64)
        u = np.zeros((3, self.n))
        lib().orc_tree_sorted(self._h, _ptr(perm), _ptr(key), _ptr(u))
        return perm, key, u

    def nodes(self):
        """Node arrays in the oracle's depth-first order, as a dict."""
        nn = self.nnodes
        d = dict(level=np.zeros(nn, np.int32), first=np.zeros(nn, np.int64),
                 count=np.zeros(nn, np.int64), parent=np.zeros(nn, np.int64),
                 nchild=np.zeros(nn, np.int32), M=np.zeros(nn), com=np.zeros((3, nn)),
                 blo=np.zeros((3, nn)), l=np.zeros(nn), rb2=np.zeros(nn))
        lib().orc_tree_nodes(self._h, *[_ptr(d[k]) for k in
                                        ("level", "first", "count", "parent", "nchild", "M",
                                         "com", "blo", "l", "rb2")])
        return d

    def set_mac(self, a_err=0.0, G=1.0, min_sinks=False):
        """Opening radii by the paper's absolute MAC (a_err > 0, section II.B)
        or l / theta (a_err = 0); groups measure cells by the minimum over
        their sinks (min_sinks) or by their bounding box."""
        lib().orc_tree_set_mac(self._h, float(a_err), float(G), int(bool(min_sinks)))
        return self

    def node_mac(self):
        """(B2, bmax2) of every node, in the order of nodes()."""
        nn = self.nnodes
        B2 = np.zeros(nn)
        bm = np.zeros(nn)
        lib().orc_tree_node_mac(self._h, _ptr(B2), _ptr(bm))
        return B2, bm

    def group_starts(self):
        """Start of each sink group in sorted order, plus n at the end."""
        s = np.zeros(self.ngroups + 1, np.int64)
        lib().orc_tree_group_starts(self._h, _ptr(s))
        return s

    def walk_counts(self, R2, hybrid):
        a = [np.zeros(self.ngroups, np.int64) for _ in range(3)]
        lib().orc_walk_counts(self._h, R2, int(hybrid), *[_ptr(v) for v in a])
        return tuple(a)

    def walk_group(self, k, R2, hybrid, cap=1 << 20):
        cnt = np.zeros(3, np.int64)
        pc = np.zeros(cap, np.int64)
        far = np.zeros(cap, np.int64)
        near = np.zeros(cap, np.int64)
        lib().orc_walk_group(self._h, k, R2, int(hybrid), cap, _ptr(pc), _ptr(far),
                             _ptr(near), _ptr(cnt))
        return pc[:cnt[0]].copy(), far[:cnt[1]].copy(), near[:cnt[2]].copy()

    def soft(self, G, eps, R1, R2, hybrid, groups=None, potential=False):
        """Soft (hybrid) or full (plain) tree force; returns (acc, pot, interactions).

        acc has shape (3, n) in caller order; sinks outside ``groups`` stay 0.
        """
        acc = np.zeros((3, self.n))
        pot = np.zeros(self.n) if potential else None
        gr = None if groups is None else np.ascontiguousarray(groups, dtype=np.int64)
        ngr = 0 if gr is None else gr.size
        inter = lib().orc_soft(self._h, G, eps, R1, R2, int(hybrid), ngr, _ptr(gr),
                               _ptr(acc), _ptr(pot))
        return acc, pot, int(inter)


def step(x, v, m, G, eps, theta, R1, R2, n_crit, g, hybrid, dt_soft, n_sub, n_soft, chunk=16):
    """Nested kick-drift-kick; returns new (x, v) (inputs are not modified).
    ``g`` and ``chunk`` set the sink groups (group size, chunking limit chunk * g)."""
    x = _f64c(x).copy()
    v = _f64c(v).copy()
    m = _f64c(m)
    lib().orc_step(x.shape[1], _ptr(x), _ptr(v), _ptr(m), G, eps, theta, R1, R2, n_crit, g,
                   int(chunk), int(hybrid), dt_soft, n_sub, n_soft)
    return x, v
