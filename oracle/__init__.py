"""CPU FP64 oracle for the Hawkes log-likelihood and gradient.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product path never imports it.

`build()` compiles oracle.c twice: single-threaded (the oracle proper) and
with OpenMP over rows (bitwise-identical results, used only to time the oracle
on all host cores and to evaluate full-size cases in tests).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB1 = os.path.join(HERE, "liboracle.so")
LIBMT = os.path.join(HERE, "liboracle_omp.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11"]

ZERORATE = -4


def build(force: bool = True) -> None:
    for out, extra in ((LIB1, []), (LIBMT, ["-fopenmp"])):
        if force or not os.path.exists(out):
            subprocess.check_call(["gcc", *CFLAGS, *extra, SRC, "-o", out, "-lm"])


_libs: dict = {}


def _lib(threads: bool):
    key = bool(threads)
    if key not in _libs:
        path = LIBMT if threads else LIB1
        if not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_loglik_grad.argtypes = [d, d, i64, ctypes.c_int, d, d, d, d]
        lib.oracle_rates.argtypes = [d, d, i64, ctypes.c_int, d, d, d]
        lib.oracle_rate_rows.argtypes = [d, d, i64, ctypes.c_int, d, ctypes.POINTER(i64), i64, d, d]
        lib.oracle_grad_rows.argtypes = [d, d, i64, ctypes.c_int, d, d, ctypes.POINTER(i64), i64, d]
        lib.oracle_grad_rows_scaled.argtypes = [d, d, i64, ctypes.c_int, d, d, ctypes.POINTER(i64), i64, d, d]
        lib.oracle_log_rates.argtypes = [d, d, i64, ctypes.c_int, d, d, d]
        lib.oracle_param_terms.argtypes = [d, d, i64, ctypes.c_int, d, d, d]
        lib.oracle_bmds.argtypes = [d, d, i64, ctypes.c_int, ctypes.c_double, d, d]
        for f in (lib.oracle_loglik_grad, lib.oracle_rates, lib.oracle_rate_rows, lib.oracle_grad_rows,
                  lib.oracle_grad_rows_scaled,
                  lib.oracle_log_rates, lib.oracle_param_terms, lib.oracle_bmds):
            f.restype = ctypes.c_int
        _libs[key] = lib
    return _libs[key]


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _prep(x, t, params):
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    t = np.ascontiguousarray(t, dtype=np.float64)
    p = np.ascontiguousarray(params, dtype=np.float64)
    assert x.shape[0] == t.shape[0] and p.shape == (6,)
    return x, t, p


def loglik_grad(x, t, params, threads: bool = False, want_grad_x: bool = True):
    """Returns (status, ll, grad_x (N,D) or None, grad_params (6,))."""
    x, t, p = _prep(x, t, params)
    n, d = x.shape
    ll = np.zeros(1)
    gx = np.zeros((n, d)) if want_grad_x else None
    gp = np.zeros(6)
    st = _lib(threads).oracle_loglik_grad(_p(x), _p(t), n, d, _p(p), _p(ll), _p(gx), _p(gp))
    return st, float(ll[0]), gx, gp


def rates(x, t, params, threads: bool = False):
    """Returns (lambda (N,), row sums (N,6) = K,R,U,J,V,W unweighted)."""
    x, t, p = _prep(x, t, params)
    n, d = x.shape
    lam = np.zeros(n)
    s6 = np.zeros((n, 6))
    st = _lib(threads).oracle_rates(_p(x), _p(t), n, d, _p(p), _p(lam), _p(s6))
    if st != 0:
        raise ValueError(f"oracle_rates status {st}")
    return lam, s6


def rate_rows(x, t, params, rows, threads: bool = True):
    """(lambda, row sums K,R,U,J,V,W) of the listed events only: the per-event
    sums of `rates`, O(N) per listed event, for spot checks of large inputs."""
    x, t, p = _prep(x, t, params)
    n, d = x.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    lam = np.zeros(rows.shape[0])
    s6 = np.zeros((rows.shape[0], 6))
    st = _lib(threads).oracle_rate_rows(_p(x), _p(t), n, d, _p(p),
                                        rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), rows.shape[0],
                                        _p(lam), _p(s6))
    if st != 0:
        raise ValueError(f"oracle_rate_rows status {st}")
    return lam, s6


def grad_rows(x, t, params, lam, rows, threads: bool = True, with_scale: bool = False):
    """Location-gradient rows (App. A) of the listed events, given every rate.
    with_scale: also each row's sum of the magnitudes of its pair
    contributions, sum_n' |c_nn'| |x_n' - x_n| (the scale of its rounding)."""
    x, t, p = _prep(x, t, params)
    n, d = x.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.zeros((rows.shape[0], d))
    sc = np.zeros(rows.shape[0]) if with_scale else None
    st = _lib(threads).oracle_grad_rows_scaled(_p(x), _p(t), n, d, _p(p), _p(lam),
                                               rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                               rows.shape[0], _p(out), _p(sc))
    if st != 0:
        raise ValueError(f"oracle_grad_rows status {st}")
    return (out, sc) if with_scale else out


def log_rates(x, t, params, threads: bool = True):
    """(log lambda (N,), largest log pair term of each row (N,)), in the log
    domain, so exact also where lambda underflows double precision."""
    x, t, p = _prep(x, t, params)
    n, d = x.shape
    ll = np.zeros(n)
    mx = np.zeros(n)
    st = _lib(threads).oracle_log_rates(_p(x), _p(t), n, d, _p(p), _p(ll), _p(mx))
    if st != 0:
        raise ValueError(f"oracle_log_rates status {st}")
    return ll, mx


def param_terms(x, t, params, threads: bool = True):
    """(sum_n v_k(n), sum_n |v_k(n)|) for the six parameter-gradient summands:
    the gradient and the cancellation scale of each component."""
    x, t, p = _prep(x, t, params)
    n, d = x.shape
    s = np.zeros(6)
    a = np.zeros(6)
    st = _lib(threads).oracle_param_terms(_p(x), _p(t), n, d, _p(p), _p(s), _p(a))
    if st != 0:
        raise ValueError(f"oracle_param_terms status {st}")
    return s, a


FLT_MIN_LOG = float(np.log(np.finfo(np.float32).tiny))


def diagnostics(x, t, params, threads: bool = True, log_floor: float = FLT_MIN_LOG):
    """The per-workload diagnostics: smallest log lambda_n, number of rows whose
    every weighted pair term lies below exp(log_floor) (by default the smallest
    normal single-precision number, so these rows have no term a plain float32
    evaluation could represent), the log-likelihood, the Frobenius norm of the
    location gradient and the parameter gradient."""
    lg, mx = log_rates(x, t, params, threads=threads)
    st, ll, gx, gp = loglik_grad(x, t, params, threads=threads)
    return {"min_log_lambda": float(lg.min()), "rows_all_terms_below_floor": int((mx < log_floor).sum()),
            "log_floor": log_floor, "status": int(st), "loglik": ll,
            "grad_x_norm": float(np.linalg.norm(gx)) if gx is not None else None,
            "grad_params": [float(v) for v in gp]}


# ---------------------------------------------------------------------------
# Per-event terms, Metropolis moves and reweighting, written from the
# definitions above (Sec. 2.1 rates; Sec. 3 location updates; Sec. 4.3
# branching probability).  Each is a plain composition of the rate and
# log-likelihood routines, so it checks the incremental GPU path against a full
# recomputation.

def event_terms(x, t, params, threads: bool = True, rows=None):
    """(N, 4): background rate per unit mu0, self-excitation rate per unit
    theta, log lambda, and theta * b / lambda (the self-excitation share of the
    rate, i.e. the probability that the event has a parent).  rows: only
    those events, in that order (O(N) each)."""
    p = np.asarray(params, dtype=np.float64)
    if rows is None:
        lam, s6 = rates(x, t, p, threads=threads)
    else:
        lam, s6 = rate_rows(x, t, p, rows, threads=threads)
    out = np.empty((lam.shape[0], 4))
    out[:, 0] = s6[:, 0]
    out[:, 1] = s6[:, 3]
    with np.errstate(divide="ignore", invalid="ignore"):
        out[:, 2] = np.log(lam)
        out[:, 3] = p[3] * s6[:, 3] / lam
    return out


def mwg_delta(x, t, params, idx, x_new, threads: bool = True):
    """Change of the log-likelihood when the events idx move to x_new: the sum
    over events of log(lambda_after / lambda_before), each rate recomputed in
    full (the compensator does not involve locations).  Returns (delta, moved x)."""
    import math
    x = np.array(x, dtype=np.float64, copy=True)
    if x.ndim == 1:
        x = x[:, None]
    lam0, _ = rates(x, t, params, threads=threads)
    x1 = x.copy()
    x1[np.asarray(idx, dtype=np.int64)] = np.asarray(x_new, dtype=np.float64).reshape(len(idx), x.shape[1])
    lam1, _ = rates(x1, t, params, threads=threads)
    with np.errstate(divide="ignore"):
        delta = math.fsum(np.log(lam1) - np.log(lam0))
    return delta, x1


def loglik_reweight(x, t, params_new, threads: bool = True):
    """(ell, d ell/d mu, d ell/d theta) at the given parameters."""
    st, ll, _, gp = loglik_grad(x, t, params_new, threads=threads, want_grad_x=False)
    return st, ll, float(gp[0]), float(gp[3])


def bmds(x, delta, sigma, threads: bool = True, want_grad_x: bool = True):
    """Bayesian MDS log-likelihood (Sec. 2.2.3): returns (status, ell,
    d ell/d sigma, pair count M, grad_x (N, D) or None).  delta is N x N; only
    the strict lower triangle is read, NaN marks an unobserved pair."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    n, d = x.shape
    assert delta.shape == (n, n)
    out = np.zeros(3)
    gx = np.zeros((n, d)) if want_grad_x else None
    st = _lib(threads).oracle_bmds(_p(x), _p(delta), n, d, float(sigma), _p(out), _p(gx))
    return st, float(out[0]), float(out[1]), float(out[2]), gx
