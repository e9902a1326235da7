"""ctypes binding of libhtree (the C ABI of include/htree.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream, every step of the force path runs in the library's kernels.  The
binding refuses to run without the built library; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "libhtree.so"

HTREE_OK = 0
HTREE_EINVAL = -1
HTREE_ENOMEM = -2
HTREE_EDEVICE = -3
HTREE_EOVERFLOW = -4
HTREE_ESTATE = -5
F_POT = 1
F_TIMING = 2
F_REUSE = 4
STATIC_SCRATCH_BYTES = 64 << 20   # HTREE_STATIC_SCRATCH_BYTES

_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EOVERFLOW", -5: "ESTATE"}


class HTreeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("htree %s: %s" % (_NAMES.get(code, code), msg))
        self.code = code


class Params(C.Structure):
    _fields_ = [("G", C.c_double), ("eps", C.c_double), ("theta", C.c_double),
                ("R1", C.c_double), ("R2", C.c_double), ("dt_soft", C.c_double),
                ("n_sub", C.c_int32), ("hybrid", C.c_int32), ("n_crit", C.c_int32),
                ("group_size", C.c_int32), ("precision", C.c_int32), ("flags", C.c_int32),
                ("group_cell", C.c_int32), ("group_mac", C.c_int32), ("a_err", C.c_double)]


class Counters(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_groups", C.c_int64), ("n_nodes", C.c_int64),
                ("n_leaves", C.c_int64), ("soft_cells", C.c_int64), ("soft_far", C.c_int64),
                ("soft_near", C.c_int64), ("soft_interactions", C.c_int64),
                ("hard_candidates", C.c_int64), ("hard_pairs", C.c_int64),
                ("ms_build", C.c_float), ("ms_soft", C.c_float), ("ms_hard", C.c_float),
                ("ms_kick", C.c_float), ("calls_build", C.c_int32), ("calls_soft", C.c_int32),
                ("calls_hard", C.c_int32), ("pad", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("failed", C.c_int64), ("cancelled", C.c_int64), ("pending", C.c_int64),
                ("in_flight", C.c_int64), ("held", C.c_int64), ("peak_in_flight", C.c_int64),
                ("arena_bytes", C.c_uint64), ("bytes_in_use", C.c_uint64),
                ("bytes_peak", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RequestInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("status", C.c_int32), ("state", C.c_int32),
                ("stream", C.c_int32), ("pad", C.c_int32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("footprint", C.c_uint64),
                ("soft_interactions", C.c_int64), ("hard_candidates", C.c_int64),
                ("hard_pairs", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_p = C.c_void_p
_st = C.c_int32


def lib() -> C.CDLL:
    """Loads libhtree.so from the package directory; raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError("libhtree.so is not built (run python -m paper_1406_6158_amd.build); "
                          "there is no non-HIP fallback")
    L = C.CDLL(str(LIB_PATH))
    L.htree_default_params.argtypes = [C.POINTER(Params)]
    L.htree_default_params.restype = None
    L.htree_workspace_bytes.argtypes = [C.POINTER(Params), C.c_int64]
    L.htree_workspace_bytes.restype = C.c_size_t
    L.htree_create.argtypes = [C.POINTER(_p), C.POINTER(Params), C.c_int64, _p, C.c_size_t, _p]
    L.htree_create_static.argtypes = [C.POINTER(_p), C.POINTER(Params), C.c_int64, _p]
    L.htree_batch_workspace_bytes.argtypes = [_p, _p, C.c_int32]
    L.htree_batch_workspace_bytes.restype = C.c_size_t
    L.htree_batch_create.argtypes = [C.POINTER(_p), _p, _p, C.c_int32, _p, C.c_size_t, _p]
    L.htree_system_count.argtypes = [_p]
    L.htree_system_count.restype = C.c_int32
    L.htree_set_state.argtypes = [_p, _p, _p, _p]
    L.htree_build_tree.argtypes = [_p]
    L.htree_soft_force.argtypes = [_p, _p, _p]
    L.htree_hard_force.argtypes = [_p, _p, _p]
    L.htree_kick_drift.argtypes = [_p, C.c_double, _p, C.c_double]
    L.htree_step.argtypes = [_p, C.c_int32]
    L.htree_refit.argtypes = [_p]
    L.htree_get_state.argtypes = [_p, _p, _p]
    L.htree_sync.argtypes = [_p]
    L.htree_stats.argtypes = [_p, C.POINTER(Counters)]
    L.htree_group_counts.argtypes = [_p, _p, _p, _p]
    L.htree_export_keys.argtypes = [_p, _p, _p, _p]
    L.htree_node_count.argtypes = [_p]
    L.htree_node_count.restype = C.c_int64
    L.htree_export_nodes.argtypes = [_p, _p, _p, _p, _p, _p]
    L.htree_export_node_mac.argtypes = [_p, _p, _p, _p]
    L.htree_export_node_boxes.argtypes = [_p, _p, _p]
    L.htree_group_count.argtypes = [_p]
    L.htree_group_count.restype = C.c_int64
    L.htree_export_groups.argtypes = [_p, _p]
    L.htree_last_error.argtypes = []
    L.htree_last_error.restype = C.c_char_p
    L.htree_destroy.argtypes = [_p]
    L.htree_destroy.restype = None
    L.htree_solve_footprint.argtypes = [C.POINTER(Params), C.c_int64]
    L.htree_solve_footprint.restype = C.c_size_t
    L.htree_server_create.argtypes = [C.POINTER(_p), _p, C.c_size_t, _p, C.c_int32, C.c_int32]
    L.htree_server_submit.argtypes = [_p, C.POINTER(Params), C.c_int64, _p, C.c_int64, _p, _p,
                                      C.POINTER(C.c_int64)]
    L.htree_server_poll.argtypes = [_p, _p, C.c_int32, C.POINTER(C.c_int32)]
    L.htree_server_result.argtypes = [_p, C.c_int64, C.POINTER(RequestInfo), C.POINTER(_p),
                                      C.POINTER(_p), C.POINTER(_p), C.POINTER(_p)]
    L.htree_server_release.argtypes = [_p, C.c_int64]
    L.htree_server_get_stats.argtypes = [_p, C.POINTER(ServerStats)]
    L.htree_server_destroy.argtypes = [_p]
    L.htree_server_destroy.restype = None
    for name in ("htree_server_create", "htree_server_submit", "htree_server_poll",
                 "htree_server_result", "htree_server_release", "htree_server_get_stats"):
        getattr(L, name).restype = _st
    for name in ("htree_create", "htree_create_static", "htree_batch_create", "htree_set_state", "htree_build_tree", "htree_soft_force",
                 "htree_hard_force", "htree_kick_drift", "htree_step", "htree_refit", "htree_get_state",
                 "htree_sync", "htree_stats", "htree_group_counts", "htree_export_keys",
                 "htree_export_nodes", "htree_export_node_mac", "htree_export_node_boxes",
                 "htree_export_groups"):
        getattr(L, name).restype = _st
    _lib = L
    return L


def check(code: int) -> None:
    if code != HTREE_OK:
        raise HTreeError(code, lib().htree_last_error().decode(errors="replace"))


def default_params(**kw) -> Params:
    p = Params()
    lib().htree_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def workspace_bytes(p: Params, n: int) -> int:
    return int(lib().htree_workspace_bytes(C.byref(p), int(n)))


def solve_footprint(p: Params, n: int) -> int:
    return int(lib().htree_solve_footprint(C.byref(p), int(n)))


def batch_arrays(params, sizes):
    """ctypes arrays (Params[S], int64[S]) for the batch entry points."""
    S = len(sizes)
    if len(params) != S:
        raise ValueError("one Params per system")
    return (Params * S)(*params), (C.c_int64 * S)(*[int(v) for v in sizes])


def batch_workspace_bytes(params, sizes) -> int:
    pa, na = batch_arrays(params, sizes)
    return int(lib().htree_batch_workspace_bytes(pa, na, len(sizes)))
