"""Thin torch-facing wrapper of the request server (htree_server_* in
include/htree.h): continuous batching of independent force solves.

torch allocates the arena (one uint8 tensor) and provides the streams; the
library queues, admits by footprint, launches and tracks the solves.  Result
tensors returned by ``result`` are views into the arena and are valid until
``release`` of that request.
"""
from __future__ import annotations

import ctypes as C

from ._abi import HTREE_OK, HTreeError, Params, RequestInfo, ServerStats, check, lib


class Server:
    """Solve server on one GPU.

    ``arena_bytes``: device memory for admitted solves (their workspaces and
    outputs); ``n_streams`` torch streams at default priority, each with up to
    ``per_stream`` solves queued on the device.
    """

    PENDING, RUNNING, DONE, FAILED = 0, 1, 2, 3

    def __init__(self, arena_bytes, n_streams=4, per_stream=2, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
            self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        handles = (C.c_void_p * n_streams)(*[s.cuda_stream for s in self.streams])
        h = C.c_void_p()
        check(lib().htree_server_create(C.byref(h), C.c_void_p(self.arena.data_ptr()),
                                        int(arena_bytes), handles, n_streams, per_stream))
        self._h = h
        self._inputs = {}      # request id -> tensors that must outlive the solve
        self._done = (C.c_int64 * 256)()

    # -- lifetime ---------------------------------------------------------------
    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().htree_server_destroy(h)
            self._h = None
            self._inputs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- ABI --------------------------------------------------------------------
    def submit(self, params: Params, x, m) -> int:
        """Queues one solve.  ``x``: float64 device tensor [3, n] whose rows
        may be strided (x[:, :n] of a larger array works); ``m``: float32 [n].
        The solve reads them after the work already enqueued on torch's
        current stream (where they are normally written)."""
        torch = self.torch
        if x.dtype != torch.float64 or x.dim() != 2 or x.shape[0] != 3 or x.stride(1) != 1:
            raise ValueError("x must be a float64 [3, n] tensor with unit column stride")
        n = int(x.shape[1])
        if m.dtype != torch.float32 or tuple(m.shape) != (n,) or not m.is_contiguous():
            raise ValueError("m must be a contiguous float32 [n] tensor")
        if x.device != self.device or m.device != self.device:
            raise ValueError("inputs must live on the server's device")
        rid = C.c_int64()
        producer = torch.cuda.current_stream(self.device).cuda_stream
        check(lib().htree_server_submit(self._h, C.byref(params), n, C.c_void_p(x.data_ptr()),
                                        int(x.stride(0)), C.c_void_p(m.data_ptr()),
                                        C.c_void_p(producer), C.byref(rid)))
        self._inputs[rid.value] = (x, m)
        return rid.value

    def poll(self):
        """Ids of requests that finished (or failed) since the last poll."""
        out = []
        nd = C.c_int32()
        while True:
            check(lib().htree_server_poll(self._h, self._done, len(self._done), C.byref(nd)))
            out.extend(self._done[k] for k in range(nd.value))
            if nd.value < len(self._done):
                return out

    def info(self, rid) -> dict:
        inf = RequestInfo()
        lib().htree_server_result(self._h, int(rid), C.byref(inf), None, None, None, None)
        return inf.as_dict()

    def result(self, rid):
        """(info, acc_soft [3,n], acc_hard [3,n] or None, ngb [n] or None,
        pot [n] or None): views into the arena, valid until release(rid).
        Raises the solve's error for a failed request."""
        torch = self.torch
        inf = RequestInfo()
        ptrs = [C.c_void_p() for _ in range(4)]
        code = lib().htree_server_result(self._h, int(rid), C.byref(inf),
                                         *[C.byref(p) for p in ptrs])
        if code != HTREE_OK:
            raise HTreeError(code, lib().htree_last_error().decode(errors="replace"))
        n = int(inf.n)
        base = self.arena.data_ptr()

        def view(p, dtype, shape, esize):
            if not p.value:
                return None
            off = p.value - base
            cnt = 1
            for s in shape:
                cnt *= s
            return self.arena[off:off + cnt * esize].view(dtype).view(*shape)

        acc_s = view(ptrs[0], torch.float32, (3, n), 4)
        acc_h = view(ptrs[1], torch.float32, (3, n), 4)
        ngb = view(ptrs[2], torch.int32, (n,), 4)
        pot = view(ptrs[3], torch.float32, (n,), 4)
        return inf.as_dict(), acc_s, acc_h, ngb, pot

    def release(self, rid):
        """Frees a finished request's block (or cancels a queued one).  Work
        that reads its result views must have completed before this call."""
        check(lib().htree_server_release(self._h, int(rid)))
        self._inputs.pop(int(rid), None)

    def stats(self) -> dict:
        st = ServerStats()
        check(lib().htree_server_get_stats(self._h, C.byref(st)))
        return st.as_dict()
