"""Python binding of the C ABI: argument marshalling only.  Every step of the
computation runs in the HIP library; torch provides device memory (the
workspace comes from torch's caching allocator) and the current HIP stream."""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from . import _lib
from ._lib import FP64, MIXED, HawkesError, HawkesParams

PRECISIONS = {"fp64": FP64, "mixed": MIXED, "fp64+cull": FP64 | _lib.CULL, "mixed+cull": MIXED | _lib.CULL,
              FP64: FP64, MIXED: MIXED, FP64 | _lib.CULL: FP64 | _lib.CULL, MIXED | _lib.CULL: MIXED | _lib.CULL}


def _prec(p) -> int:
    """'fp64' or 'mixed', optionally with '+cull' (exact culling of tiles whose
    pair terms all underflow; bitwise the same results)."""
    try:
        return PRECISIONS[p]
    except KeyError:
        raise ValueError(f"precision must be 'fp64', 'mixed', 'fp64+cull' or 'mixed+cull', got {p!r}")


def params_struct(params: Sequence[float]) -> HawkesParams:
    p = [float(v) for v in (params.tolist() if hasattr(params, "tolist") else params)]
    if len(p) != 6:
        raise ValueError("params must have 6 entries (mu, h, tau, theta, omega, xi)")
    return HawkesParams(*p)


def workspace_bytes(n: int, d: int, prec="mixed") -> int:
    return int(_lib.lib().hawkes_workspace_bytes(int(n), int(d), _prec(prec)))


_ws_cache: dict = {}


def workspace(n: int, d: int, prec, device) -> torch.Tensor:
    """Cached workspace, one per device and stream: calls on one stream run in
    order, so they can share it (a stream must not be driven from two threads
    at once).  It is allocated on that stream, so torch's caching allocator
    only hands it out again behind the work queued there."""
    need = workspace_bytes(n, d, prec)
    if need == 0:
        raise HawkesError(_lib.EINVAL, "workspace size")
    dev = torch.device(device)
    key = (dev, _stream_ptr(dev))
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        _ws_cache[key] = ws
    return ws


def _check_inputs(x: torch.Tensor, t: torch.Tensor):
    if not (x.is_cuda and t.is_cuda):
        raise ValueError("x and t must be device tensors")
    if x.dtype != torch.float64 or t.dtype != torch.float64:
        raise ValueError("x and t must be float64")
    if x.dim() != 2 or t.dim() != 1 or x.shape[0] != t.shape[0]:
        raise ValueError("x must be (N, D) and t (N,)")
    return x.contiguous(), t.contiguous()


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def loglik(x: torch.Tensor, t: torch.Tensor, params, prec="mixed") -> float:
    x, t = _check_inputs(x, t)
    n, d = x.shape
    ws = workspace(n, d, prec, x.device)
    ll = ctypes.c_double(0.0)
    ps = params_struct(params)
    st = _lib.lib().hawkes_loglik(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), _prec(prec), ws.data_ptr(),
                                  ws.numel(), _stream_ptr(x.device), ctypes.byref(ll))
    if st not in (_lib.OK, _lib.EZERORATE):
        raise HawkesError(st, "hawkes_loglik")
    return ll.value


def grad(x: torch.Tensor, t: torch.Tensor, params, prec="mixed", out: torch.Tensor | None = None,
         raise_zero_rate: bool = False):
    """Returns (loglik, grad_x (N, D) float64 device tensor, grad_params numpy (6,))."""
    x, t = _check_inputs(x, t)
    n, d = x.shape
    ws = workspace(n, d, prec, x.device)
    gx = out if out is not None else torch.empty_like(x)
    ll = ctypes.c_double(0.0)
    gp = (ctypes.c_double * 6)()
    ps = params_struct(params)
    st = _lib.lib().hawkes_grad(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), _prec(prec), ws.data_ptr(),
                                ws.numel(), _stream_ptr(x.device), ctypes.byref(ll), gx.data_ptr(), gp)
    if st != _lib.OK and (st != _lib.EZERORATE or raise_zero_rate):
        raise HawkesError(st, "hawkes_grad")
    return ll.value, gx, np.array(gp[:])


def grad_async(x: torch.Tensor, t: torch.Tensor, params, prec="mixed", out8: torch.Tensor | None = None,
               grad_x: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """Enqueue a full evaluation on the current stream without synchronizing.
    out8 (device, 8 doubles) receives [loglik, 6 parameter gradients, status]."""
    x, t = _check_inputs(x, t)
    n, d = x.shape
    if ws is None:
        ws = workspace(n, d, prec, x.device)
    if out8 is None:
        out8 = torch.empty(8, dtype=torch.float64, device=x.device)
    ps = params_struct(params)
    st = _lib.lib().hawkes_grad_async(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), _prec(prec),
                                      ws.data_ptr(), ws.numel(), _stream_ptr(x.device), out8.data_ptr(),
                                      grad_x.data_ptr() if grad_x is not None else None)
    if st != _lib.OK:
        raise HawkesError(st, "hawkes_grad_async")
    return out8


def event_terms(x: torch.Tensor, t: torch.Tensor, params, prec="fp64", out: torch.Tensor | None = None):
    """Per-event terms (device (N, 4) float64: background rate per unit mu0,
    self-excitation rate per unit theta, log lambda, branching probability)
    and the log-likelihood.  Synchronizes the current stream."""
    x, t = _check_inputs(x, t)
    n, d = x.shape
    ws = workspace(n, d, prec, x.device)
    terms = out if out is not None else torch.empty((n, 4), dtype=torch.float64, device=x.device)
    ll = ctypes.c_double(0.0)
    ps = params_struct(params)
    st = _lib.lib().hawkes_event_terms(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), _prec(prec),
                                       ws.data_ptr(), ws.numel(), _stream_ptr(x.device), terms.data_ptr(),
                                       ctypes.byref(ll))
    if st not in (_lib.OK, _lib.EZERORATE):
        raise HawkesError(st, "hawkes_event_terms")
    return terms, ll.value


def diagnostics(x: torch.Tensor, t: torch.Tensor, params, prec="mixed"):
    """Which rows the float64 fix-up recomputed in the last evaluation of
    (x, t, params, prec) on the current stream (the cached workspace of
    loglik / grad / grad_async / event_terms).  Returns (dict of the
    diagnostics fields, flags as a numpy int32 array (N,)).  Synchronizes."""
    x, t = _check_inputs(x, t)
    n, d = x.shape
    ws = workspace(n, d, prec, x.device)
    flags = torch.empty(n, dtype=torch.int32, device=x.device)
    out = _lib.HawkesDiag()
    ps = params_struct(params)
    st = _lib.lib().hawkes_diagnostics(ws.data_ptr(), ws.numel(), n, d, _prec(prec), ctypes.byref(ps),
                                       _stream_ptr(x.device), flags.data_ptr(), ctypes.byref(out))
    if st != _lib.OK:
        raise HawkesError(st, "hawkes_diagnostics")
    info = {k: getattr(out, k) for k, _ in _lib.HawkesDiag._fields_}
    return info, flags.cpu().numpy()


_mwg_ws: dict = {}


def mwg_workspace(n: int, device) -> torch.Tensor:
    """Cached Metropolis-within-Gibbs workspace, one per device and stream."""
    need = int(_lib.lib().hawkes_mwg_workspace_bytes(int(n)))
    if need == 0:
        raise HawkesError(_lib.EINVAL, "mwg workspace size")
    dev = torch.device(device)
    key = (dev, _stream_ptr(dev))
    ws = _mwg_ws.get(key)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        _mwg_ws[key] = ws
    return ws


def mwg_step(x: torch.Tensor, t: torch.Tensor, params, terms: torch.Tensor, idx: torch.Tensor,
             x_new: torch.Tensor, log_thresh: torch.Tensor, out3: torch.Tensor | None = None,
             ws: torch.Tensor | None = None) -> torch.Tensor:
    """Enqueue one Metropolis step moving events idx (device int64, strictly
    increasing) to x_new; x and terms are updated in place on accept.
    Returns out3 (device): [Delta loglik, accepted, status]."""
    if not (x.is_contiguous() and terms.is_contiguous() and x.dtype == torch.float64):
        raise ValueError("x and terms must be contiguous float64 device tensors")
    if idx.dtype != torch.int64 or x_new.dtype != torch.float64 or log_thresh.dtype != torch.float64:
        raise ValueError("idx must be int64, x_new and log_thresh float64")
    n, d = x.shape
    if terms.shape != (n, 4) or x_new.shape != (idx.numel(), d) or log_thresh.numel() < 1:
        raise ValueError("shape mismatch")
    idx, x_new = idx.contiguous(), x_new.contiguous()
    if ws is None:
        ws = mwg_workspace(n, x.device)
    if out3 is None:
        out3 = torch.empty(3, dtype=torch.float64, device=x.device)
    ps = params_struct(params)
    st = _lib.lib().hawkes_mwg_step(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), terms.data_ptr(),
                                    idx.data_ptr(), x_new.data_ptr(), idx.numel(), log_thresh.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _stream_ptr(x.device), out3.data_ptr())
    if st != _lib.OK:
        raise HawkesError(st, "hawkes_mwg_step")
    return out3


def loglik_reweight(t: torch.Tensor, d: int, params, terms: torch.Tensor,
                    out3: torch.Tensor | None = None) -> torch.Tensor:
    """Enqueue ell and its mu/theta derivatives at new weights from cached
    terms (every other parameter as when the terms were computed)."""
    n = t.numel()
    if terms.shape != (n, 4) or not terms.is_contiguous():
        raise ValueError("terms must be a contiguous (N, 4) tensor")
    if out3 is None:
        out3 = torch.empty(3, dtype=torch.float64, device=t.device)
    ps = params_struct(params)
    st = _lib.lib().hawkes_loglik_reweight(t.data_ptr(), n, d, ctypes.byref(ps), terms.data_ptr(),
                                           _stream_ptr(t.device), out3.data_ptr())
    if st != _lib.OK:
        raise HawkesError(st, "hawkes_loglik_reweight")
    return out3


_BOUNDS = {None: _lib.BOUND_NONE, "none": _lib.BOUND_NONE, "box": _lib.BOUND_BOX, "disc": _lib.BOUND_DISC}


def _trajectory_args(x, p, t, bound, b0, b1, grad_x, have_grad, out8):
    if not (x.is_contiguous() and p.is_contiguous() and x.dtype == torch.float64 and p.dtype == torch.float64):
        raise ValueError("x and p must be contiguous float64 device tensors")
    n, d = x.shape
    if p.shape != x.shape or t.shape != (n,):
        raise ValueError("shape mismatch")
    kind = _BOUNDS[bound]
    if kind != _lib.BOUND_NONE:
        if b0 is None or b1 is None:
            raise ValueError("bounds need b0 and b1")
        b0, b1 = b0.contiguous(), b1.contiguous()
        want1 = (n, d) if kind == _lib.BOUND_BOX else (n,)
        if b0.shape != (n, d) or b1.shape != want1:
            raise ValueError("bound shape mismatch")
    if grad_x is None:
        grad_x = torch.empty_like(x)
        have_grad = False
    if out8 is None:
        out8 = torch.empty(8, dtype=torch.float64, device=x.device)
    return n, d, kind, b0, b1, grad_x, have_grad, out8


def leapfrog(x: torch.Tensor, p: torch.Tensor, t: torch.Tensor, params, eps: float, steps: int, prec="mixed",
             bound=None, b0: torch.Tensor | None = None, b1: torch.Tensor | None = None,
             grad_x: torch.Tensor | None = None, have_grad: bool = False, out8: torch.Tensor | None = None):
    """Enqueue `steps` leapfrog steps on the current stream; x and p (device
    (N, D) float64, contiguous) move in place.  bound: None, "box" (b0/b1 =
    lower/upper corners) or "disc" (b0 = centres, b1 = radii).  Returns
    (grad_x at the final x, out8 = [loglik, 6 parameter gradients, status])."""
    n, d, kind, b0, b1, grad_x, have_grad, out8 = _trajectory_args(x, p, t, bound, b0, b1, grad_x, have_grad, out8)
    ws = workspace(n, d, prec, x.device)
    ps = params_struct(params)
    st = _lib.lib().hawkes_leapfrog(x.data_ptr(), p.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), _prec(prec),
                                    float(eps), int(steps), kind, b0.data_ptr() if b0 is not None else None,
                                    b1.data_ptr() if b1 is not None else None, ws.data_ptr(), ws.numel(),
                                    _stream_ptr(x.device), grad_x.data_ptr(), 1 if have_grad else 0,
                                    out8.data_ptr())
    if st != _lib.OK:
        raise HawkesError(st, "hawkes_leapfrog")
    return grad_x, out8


def leapfrog_bmds(x: torch.Tensor, p: torch.Tensor, t: torch.Tensor, params, delta: torch.Tensor, sigma: float,
                  eps: float, steps: int, prec="mixed", bound=None, b0: torch.Tensor | None = None,
                  b1: torch.Tensor | None = None, grad_x: torch.Tensor | None = None, have_grad: bool = False,
                  out8: torch.Tensor | None = None, out4: torch.Tensor | None = None):
    """As `leapfrog`, for the influenza model's joint potential
    -(Hawkes log-likelihood + MDS log-likelihood of delta): returns (grad_x,
    out8 of the final Hawkes evaluation, out4 of the final MDS evaluation)."""
    n, d, kind, b0, b1, grad_x, have_grad, out8 = _trajectory_args(x, p, t, bound, b0, b1, grad_x, have_grad, out8)
    if delta.dtype != torch.float64 or delta.shape != (n, n) or not delta.is_contiguous():
        raise ValueError("delta must be a contiguous (N, N) float64 device tensor")
    if out4 is None:
        out4 = torch.empty(4, dtype=torch.float64, device=x.device)
    ws = workspace(n, d, prec, x.device)
    bws = _bmds_workspace(n, d, x.device)
    ps = params_struct(params)
    st = _lib.lib().hawkes_leapfrog_bmds(x.data_ptr(), p.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps),
                                         _prec(prec), delta.data_ptr(), float(sigma), float(eps), int(steps), kind,
                                         b0.data_ptr() if b0 is not None else None,
                                         b1.data_ptr() if b1 is not None else None, ws.data_ptr(), ws.numel(),
                                         bws.data_ptr(), bws.numel(), _stream_ptr(x.device), grad_x.data_ptr(),
                                         1 if have_grad else 0, out8.data_ptr(), out4.data_ptr())
    if st != _lib.OK:
        raise HawkesError(st, "hawkes_leapfrog_bmds")
    return grad_x, out8, out4


_bmds_ws: dict = {}


def _bmds_workspace(n: int, d: int, device):
    """MDS workspace for (n, d) on `device`, kept per (device, stream)."""
    need = int(_lib.lib().hawkes_bmds_workspace_bytes(n, d))
    if need == 0:
        raise HawkesError(_lib.EINVAL, "bmds workspace size")
    key = (device, _stream_ptr(device))
    ws = _bmds_ws.get(key)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
        _bmds_ws[key] = ws
    return ws


def bmds(x: torch.Tensor, delta: torch.Tensor, sigma: float, prec="fp64", grad_x: torch.Tensor | None = None,
         want_grad: bool = True, out4: torch.Tensor | None = None):
    """Enqueue the Bayesian MDS log-likelihood on the current stream.  x: (N, D)
    float64 device; delta: (N, N) float64 device (strict lower triangle read,
    NaN = unobserved).  Returns (out4 = [loglik, d/d sigma, pairs, status],
    grad_x or None)."""
    if x.dtype != torch.float64 or delta.dtype != torch.float64:
        raise ValueError("x and delta must be float64")
    x, delta = x.contiguous(), delta.contiguous()
    n, d = x.shape
    if delta.shape != (n, n):
        raise ValueError("delta must be (N, N)")
    ws = _bmds_workspace(n, d, x.device)
    if want_grad and grad_x is None:
        grad_x = torch.empty_like(x)
    if out4 is None:
        out4 = torch.empty(4, dtype=torch.float64, device=x.device)
    st = _lib.lib().hawkes_bmds(x.data_ptr(), delta.data_ptr(), n, d, float(sigma), _prec(prec), ws.data_ptr(),
                                ws.numel(), _stream_ptr(x.device), out4.data_ptr(),
                                grad_x.data_ptr() if want_grad else None)
    if st != _lib.OK:
        raise HawkesError(st, "hawkes_bmds")
    return out4, (grad_x if want_grad else None)
