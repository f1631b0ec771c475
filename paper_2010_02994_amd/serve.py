"""Client of the continuous-batching server (C ABI hawkes_serve_*).

The server runs in the library: a native scheduler thread admits requests by
free slots and HBM footprint and launches batches on several HIP streams.
This class only marshals arguments and keeps the client's device buffers alive
until their requests complete.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import HawkesError, ServeResult, ServeStats
from .api import _prec, params_struct


class _TorchMemory:
    """Device memory for a server from PyTorch's caching allocator: each block
    is a uint8 tensor kept alive until the server gives the pointer back."""

    def __init__(self, device):
        self.device = device
        self.blocks: dict[int, object] = {}
        self._alloc = _lib.ALLOC_FN(self._on_alloc)
        self._free = _lib.FREE_FN(self._on_free)
        self.spec = _lib.HawkesAllocator(self._alloc, self._free, None)

    def _on_alloc(self, nbytes, ctx):
        try:
            import torch
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except Exception:   # out of memory: the server reports the failure
            return None
        self.blocks[t.data_ptr()] = t
        return t.data_ptr()

    def _on_free(self, ptr, ctx):
        self.blocks.pop(int(ptr), None)


class Server:
    def __init__(self, hbm_budget_bytes: int = 8 << 30, max_slots: int = 64, streams: int = 2,
                 simulate: bool = False, torch_memory: bool = False, device="cuda:0"):
        """torch_memory: take the server's device buffers from PyTorch's
        caching allocator (hawkes_serve_create_with) instead of hipMalloc."""
        self._L = _lib.lib()
        self._h = ctypes.c_void_p()
        flags = (streams & 0xFF) | (_lib.SERVE_SIMULATE if simulate else 0)
        self._mem = _TorchMemory(device) if torch_memory else None
        if self._mem is not None:
            st = self._L.hawkes_serve_create_with(ctypes.byref(self._mem.spec), int(hbm_budget_bytes),
                                                  int(max_slots), flags, ctypes.byref(self._h))
        else:
            st = self._L.hawkes_serve_create(int(hbm_budget_bytes), int(max_slots), flags, ctypes.byref(self._h))
        if st != _lib.OK:
            raise HawkesError(st, "hawkes_serve_create")
        self.simulate = simulate
        self._keep: dict[int, tuple] = {}
        self._datasets: dict[int, tuple] = {}

    @staticmethod
    def footprint(n: int, d: int, prec="mixed") -> int:
        return int(_lib.lib().hawkes_serve_footprint(int(n), int(d), _prec(prec)))

    def register(self, t, d: int, n: int | None = None) -> int:
        """t: device float64 tensor of sorted times (or, in simulate mode, any
        object with a data pointer).  Returns the dataset id."""
        ptr = t.data_ptr() if hasattr(t, "data_ptr") else int(t)
        n = int(t.shape[0]) if n is None else int(n)
        ds = ctypes.c_int32()
        st = self._L.hawkes_serve_register(self._h, ptr, n, int(d), ctypes.byref(ds))
        if st != _lib.OK:
            raise HawkesError(st, "hawkes_serve_register")
        self._datasets[ds.value] = (t, n, int(d))
        return ds.value

    def submit(self, dataset: int, x, params, prec="mixed", grad_x=None) -> int:
        xp = x.data_ptr() if hasattr(x, "data_ptr") else int(x)
        gp = (grad_x.data_ptr() if hasattr(grad_x, "data_ptr") else int(grad_x)) if grad_x is not None else None
        ps = params_struct(params)
        tk = ctypes.c_uint64()
        st = self._L.hawkes_serve_submit(self._h, int(dataset), xp, ctypes.byref(ps), _prec(prec), gp,
                                         ctypes.byref(tk))
        if st != _lib.OK:
            raise HawkesError(st, "hawkes_serve_submit")
        self._keep[tk.value] = (x, grad_x)
        return tk.value

    @staticmethod
    def _res(r: ServeResult) -> dict:
        return {"status": r.status, "loglik": r.loglik, "grad_params": list(r.grad_params),
                "t_submit_ns": r.t_submit_ns, "t_admit_ns": r.t_admit_ns, "t_start_ns": r.t_start_ns,
                "t_done_ns": r.t_done_ns}

    def poll(self, ticket: int):
        r = ServeResult()
        st = self._L.hawkes_serve_poll(self._h, int(ticket), ctypes.byref(r))
        if st == _lib.EPENDING:
            return None
        if st != _lib.OK:
            raise HawkesError(st, "hawkes_serve_poll")
        self._keep.pop(ticket, None)
        return self._res(r)

    def wait(self, ticket: int, timeout_s: float | None = None) -> dict:
        r = ServeResult()
        to = -1 if timeout_s is None else int(timeout_s * 1e9)
        st = self._L.hawkes_serve_wait(self._h, int(ticket), ctypes.byref(r), to)
        if st != _lib.OK:
            raise HawkesError(st, "hawkes_serve_wait")
        self._keep.pop(ticket, None)
        return self._res(r)

    def stats(self) -> dict:
        s = ServeStats()
        st = self._L.hawkes_serve_stats(self._h, ctypes.byref(s))
        if st != _lib.OK:
            raise HawkesError(st, "hawkes_serve_stats")
        return {k: getattr(s, k) for k, _ in ServeStats._fields_}

    def device_blocks(self) -> int:
        """Device buffers the server holds from PyTorch (torch_memory only)."""
        return len(self._mem.blocks) if self._mem is not None else 0

    def close(self):
        if self._h:
            self._L.hawkes_serve_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
