"""MI355X (gfx950) library for the force path of the hybrid hard/soft tree
method for collision-less N-body systems (Watanabe & Nakasato,
arXiv:1406.6158): octree soft force, neighbour-search hard force and the
two-timestep leapfrog, behind the C ABI of include/htree.h.

``HTree`` is a thin torch-facing wrapper: torch allocates the device
workspace and provides the stream; all computation happens in libhtree's HIP
kernels.
"""
from __future__ import annotations

import ctypes as C

from ._abi import (F_POT, F_TIMING, F_REUSE, STATIC_SCRATCH_BYTES, HTREE_EINVAL, HTREE_ENOMEM, HTREE_EOVERFLOW, HTREE_ESTATE,
                   HTreeError, Params, Counters, batch_arrays, batch_workspace_bytes, check,
                   default_params, lib, solve_footprint, workspace_bytes)
from .server import Server

__all__ = ["HTree", "Server", "solve_footprint", "Params", "Counters", "HTreeError", "default_params", "workspace_bytes",
           "batch_workspace_bytes", "lib", "F_POT", "F_TIMING", "F_REUSE", "STATIC_SCRATCH_BYTES", "HTREE_EINVAL", "HTREE_ENOMEM",
           "HTREE_EOVERFLOW", "HTREE_ESTATE"]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class HTree:
    """One particle system, or a batch of independent systems, on one GPU.

    ``params`` is a ``Params`` (see ``default_params``) and ``n`` the particle
    count; for a batch, ``params`` is a list with one ``Params`` per system and
    ``n`` the list of their sizes (arrays then concatenate the systems in
    order).  The workspace is a torch uint8 tensor on ``device``; calls are
    enqueued on ``stream`` (default: torch's current stream at construction).
    ``static=True`` (one system only) uses the library's static device scratch
    instead (htree_create_static): nothing is allocated for the workspace.
    """

    def __init__(self, n, params, device="cuda", stream=None, static=False):
        import torch
        self.torch = torch
        self.batch = isinstance(n, (list, tuple))
        self.sizes = [int(v) for v in n] if self.batch else [int(n)]
        self.n = sum(self.sizes)
        self.params = params
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream()
            if static:
                if self.batch:
                    raise ValueError("the static scratch serves one system")
                h = C.c_void_p()
                self.nbytes = 0
                self.workspace = None
                check(lib().htree_create_static(C.byref(h), C.byref(params), self.n,
                                                C.c_void_p(self.stream.cuda_stream)))
                self._h = h
                return
            if self.batch:
                pa, na = batch_arrays(params, self.sizes)
                nbytes = int(lib().htree_batch_workspace_bytes(pa, na, len(self.sizes)))
            else:
                nbytes = workspace_bytes(params, self.n)
            if nbytes == 0:
                raise HTreeError(HTREE_EINVAL, lib().htree_last_error().decode())
            self.nbytes = nbytes
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            h = C.c_void_p()
            if self.batch:
                check(lib().htree_batch_create(C.byref(h), pa, na, len(self.sizes),
                                               C.c_void_p(self.workspace.data_ptr()), nbytes,
                                               C.c_void_p(self.stream.cuda_stream)))
            else:
                check(lib().htree_create(C.byref(h), C.byref(params), self.n,
                                         C.c_void_p(self.workspace.data_ptr()), nbytes,
                                         C.c_void_p(self.stream.cuda_stream)))
        self._h = h

    @property
    def group_size(self):
        return (self.params[0] if self.batch else self.params).group_size

    # -- lifetime ---------------------------------------------------------------
    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self.sync_stream()
            lib().htree_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def sync_stream(self):
        self.stream.synchronize()

    # -- helpers ----------------------------------------------------------------
    def _dev(self, t, dtype, shape):
        torch = self.torch
        t = torch.as_tensor(t)
        t = t.to(device=self.device, dtype=dtype).contiguous()
        if tuple(t.shape) != shape:
            raise ValueError("expected shape %s, got %s" % (shape, tuple(t.shape)))
        return t

    def _new(self, dtype, shape):
        return self.torch.empty(shape, dtype=dtype, device=self.device)

    # -- ABI --------------------------------------------------------------------
    def set_state(self, x, v, m):
        torch = self.torch
        n = self.n
        self._x = self._dev(x, torch.float64, (3, n))
        self._v = None if v is None else self._dev(v, torch.float32, (3, n))
        self._m = self._dev(m, torch.float32, (n,))
        check(lib().htree_set_state(self._h, _ptr(self._x), _ptr(self._v), _ptr(self._m)))
        return self

    def build_tree(self):
        check(lib().htree_build_tree(self._h))
        return self

    def soft_force(self, out=None, pot=None, want_pot=False):
        torch = self.torch
        if out is None:
            out = self._new(torch.float32, (3, self.n))
        if want_pot and pot is None:
            pot = self._new(torch.float32, (self.n,))
        check(lib().htree_soft_force(self._h, _ptr(out), _ptr(pot)))
        return (out, pot) if want_pot else out

    def hard_force(self, out=None, ngb=None):
        torch = self.torch
        if out is None:
            out = self._new(torch.float32, (3, self.n))
        if ngb is None:
            ngb = self._new(torch.int32, (self.n,))
        check(lib().htree_hard_force(self._h, _ptr(out), _ptr(ngb)))
        return out, ngb

    def kick_drift(self, dt_kick, acc=None, dt_drift=0.0):
        a = None if acc is None else self._dev(acc, self.torch.float32, (3, self.n))
        check(lib().htree_kick_drift(self._h, float(dt_kick), _ptr(a), float(dt_drift)))
        self._keep = a
        return self

    def refit(self):
        check(lib().htree_refit(self._h))
        return self

    def step(self, n_soft_steps=1):
        check(lib().htree_step(self._h, int(n_soft_steps)))
        return self

    def get_state(self):
        torch = self.torch
        x = self._new(torch.float64, (3, self.n))
        v = self._new(torch.float32, (3, self.n))
        check(lib().htree_get_state(self._h, _ptr(x), _ptr(v)))
        return x, v

    def sync(self):
        check(lib().htree_sync(self._h))

    def stats(self) -> dict:
        c = Counters()
        check(lib().htree_stats(self._h, C.byref(c)))
        return c.as_dict()

    def group_starts(self):
        import numpy as np
        ng = int(lib().htree_group_count(self._h))
        if ng < 0:
            check(-5)
        s = np.zeros(ng + 1, np.int32)
        check(lib().htree_export_groups(self._h, C.c_void_p(s.ctypes.data)))
        return s

    def group_counts(self):
        import numpy as np
        ng = int(lib().htree_group_count(self._h))
        a = [np.zeros(ng, np.int32) for _ in range(3)]
        check(lib().htree_group_counts(self._h, *[C.c_void_p(v.ctypes.data) for v in a]))
        return tuple(a)

    def export_keys(self):
        import numpy as np
        keys = np.zeros(self.n, np.uint64)
        perm = np.zeros(self.n, np.int32)
        fr = np.zeros(4 * len(self.sizes))
        check(lib().htree_export_keys(self._h, C.c_void_p(keys.ctypes.data),
                                      C.c_void_p(perm.ctypes.data), C.c_void_p(fr.ctypes.data)))
        if self.batch:
            fr = fr.reshape(-1, 4)
            return keys, perm, fr[:, :3].copy(), fr[:, 3].copy()
        return keys, perm, fr[:3].copy(), float(fr[3])

    def export_nodes(self):
        import numpy as np
        nn = int(lib().htree_node_count(self._h))
        if nn < 0:
            check(-3)
        d = dict(level=np.zeros(nn, np.int32), first=np.zeros(nn, np.int32),
                 count=np.zeros(nn, np.int32), M=np.zeros(nn), com=np.zeros((3, nn)))
        check(lib().htree_export_nodes(self._h, *[C.c_void_p(d[k].ctypes.data) for k in
                                                  ("level", "first", "count", "M", "com")]))
        return d

    def export_node_boxes(self):
        """(lo, hi) [3][nn] bounding boxes of the nodes' particles at the
        positions of the last build or refit, in export_nodes order."""
        import numpy as np
        nn = int(lib().htree_node_count(self._h))
        if nn < 0:
            check(-3)
        lo, hi = np.zeros((3, nn)), np.zeros((3, nn))
        check(lib().htree_export_node_boxes(self._h, C.c_void_p(lo.ctypes.data),
                                            C.c_void_p(hi.ctypes.data)))
        return lo, hi

    def export_node_mac(self):
        """(B2, bmax2, rb2) of the last build's nodes, in export_nodes order."""
        import numpy as np
        nn = int(lib().htree_node_count(self._h))
        if nn < 0:
            check(-3)
        a = [np.zeros(nn) for _ in range(3)]
        check(lib().htree_export_node_mac(self._h, *[C.c_void_p(v.ctypes.data) for v in a]))
        return tuple(a)
