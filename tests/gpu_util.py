"""Helpers shared by the GPU parity tests (comparison metrics and runners)."""
import sys

import numpy as np

TOL = {"fp64": {"ll": 1e-10, "gx": 1e-10, "gp": 1e-10},
       "mixed": {"ll": 1e-5, "gx": 1e-4, "gp": 1e-4}}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(w_x, w_t, params, prec):
    import torch
    from paper_2010_02994_amd import api
    x = torch.tensor(np.ascontiguousarray(w_x), device="cuda:0")
    t = torch.tensor(np.ascontiguousarray(w_t), device="cuda:0")
    ll, gx, gp = api.grad(x, t, params, prec=prec)
    torch.cuda.synchronize()
    return ll, gx.cpu().numpy(), gp


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def rel_norm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def param_err(gp, gp_ref, params, n):
    """Largest |theta_k (g_k - g*_k)| over the natural scale max(|theta (.) g*|, N):
    theta_k dl/dtheta_k sums O(1) per-event terms, so N is its cancellation scale."""
    params = np.asarray(params)
    scale = max(float(np.linalg.norm(params * gp_ref)), float(n))
    return float(np.max(np.abs(params * (gp - gp_ref))) / scale)


def check(prec, ll, gx, gp, ll_ref, gx_ref, gp_ref, params, n, label=""):
    tol = TOL[prec]
    e_ll = rel(ll, ll_ref)
    e_gx = rel_norm(gx, gx_ref) if gx_ref is not None else 0.0
    e_gp = param_err(gp, gp_ref, params, n)
    say(f"  {label} {prec}: ll {ll:.15g} ref {ll_ref:.15g} | err ll {e_ll:.2e} gx {e_gx:.2e} gp {e_gp:.2e}")
    assert e_ll <= tol["ll"], f"loglik rel err {e_ll}"
    assert e_gx <= tol["gx"], f"grad_x rel err {e_gx}"
    assert e_gp <= tol["gp"], f"grad_params err {e_gp}"
    return e_ll, e_gx, e_gp
