"""Helpers shared by the GPU parity tests: oracle references, the comparison
metrics and the runners.

Metrics (each against the float64 oracle):
  ll   |l - l*| / |l*|
  gx   ||G - G*||_F / ||G*||_F over the compared rows
  row  the worst row: max_n ||g_n - g*_n|| / s_n, where s_n is the oracle's sum
       of the magnitudes of row n's pair contributions, sum_n' |c_nn'| |x_n' - x_n|
       (the size against which any evaluation of row n rounds; a row with
       s_n = 0 has no active pair and must come out exactly zero)
  gp   ||Theta (.) (g - g*)|| / ||Theta (.) g*|| (the dimensionless parameter gradient)
  gpk  max_k |g_k - g*_k| / A_k, A_k = sum_n |v_k(n)| the cancellation scale of
       parameter-gradient component k (v_k(n): event n's summand)

Tolerances: float64 1e-10 for every metric.  Mixed: 1e-5 (ll) and 1e-4 (gx,
gp) as the precision contract states; for the per-row and per-component
metrics, which no averaging over rows helps, the bound follows from the
float32 pair arithmetic: locations are rounded to float32 in units of the
spatial bandwidth, as offsets from the data's centre, so with locations
spanning up to ~250 bandwidths (the 500 km box) each coordinate difference
carries an absolute error up to ulp(250) = 1.5e-5 bandwidths and a pair term a
relative error up to ~1e-4 (that error times the exponent's slope, ~2|dx|, at
the distances where terms matter); times are offsets from each column tile's
first event, exact to ~2^-24 of the pair's time difference.  A row's or a
component's error is a weighted mean of its terms' errors, so it stays below
3e-4 of its scale."""
import dataclasses
import sys

import numpy as np

TOL = {"fp64": {"ll": 1e-10, "gx": 1e-10, "gp": 1e-10, "row": 1e-10, "gpk": 1e-10},
       "mixed": {"ll": 1e-5, "gx": 1e-4, "gp": 1e-4, "row": 3e-4, "gpk": 3e-4}}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@dataclasses.dataclass
class Ref:
    """Oracle reference of one evaluation."""
    ll: float
    gp: np.ndarray               # (6,) parameter gradient
    gp_scale: np.ndarray         # (6,) A_k
    gx: np.ndarray | None = None          # (len(rows), D) location-gradient rows
    rows: np.ndarray | None = None        # their indices (None: every row, in order)
    row_scale: np.ndarray | None = None   # (len(rows),) s_n


def oracle_ref(x, t, params, rows=None, want_gx=True) -> Ref:
    """The oracle's log-likelihood, parameter gradient with its per-component
    cancellation scales, and (want_gx) the location-gradient rows `rows` (all
    when None) with their per-row scales; threaded C oracle."""
    import oracle
    st, ll, _, _ = oracle.loglik_grad(x, t, params, threads=True, want_grad_x=False)
    assert st == 0, st
    gp, a6 = oracle.param_terms(x, t, params)
    ref = Ref(ll=ll, gp=gp, gp_scale=a6)
    if want_gx:
        lam, _ = oracle.rates(x, t, params, threads=True)
        r = np.arange(len(t)) if rows is None else np.asarray(rows)
        ref.gx, ref.row_scale = oracle.grad_rows(x, t, params, lam, r, with_scale=True)
        ref.rows = None if rows is None else r
    return ref


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


def param_errors(gp, ref: Ref, params):
    """(relative norm of Theta (.) dg, worst component against A_k, its index)."""
    p = np.asarray(params, dtype=np.float64)
    d = np.asarray(gp) - ref.gp
    e_norm = float(np.linalg.norm(p * d) / max(np.linalg.norm(p * ref.gp), 1e-300))
    per = np.abs(d) / np.maximum(ref.gp_scale, 1e-300)
    k = int(np.argmax(per))
    return e_norm, float(per[k]), k


def row_errors(gx_rows, ref: Ref):
    """(worst ||dg_n|| / s_n, its row index, that row's error relative to its
    own norm).  Rows with s_n = 0 must be exactly zero (error inf otherwise)."""
    d = np.linalg.norm(gx_rows - ref.gx, axis=1)
    s = ref.row_scale
    per = np.where(s > 0, d / np.where(s > 0, s, 1.0), np.where(d == 0, 0.0, np.inf))
    j = int(np.argmax(per))
    own = float(d[j] / max(np.linalg.norm(ref.gx[j]), 1e-300))
    row = int(j if ref.rows is None else ref.rows[j])
    return float(per[j]), row, own


def check(prec, got, ref: Ref, params, label=""):
    """Compare one GPU evaluation (ll, grad_x (N, D) or None, grad_params) with
    the oracle reference at the precision's tolerances; prints every metric."""
    ll, gx, gp = got
    tol = TOL[prec.split("+")[0]]
    e_ll = rel(ll, ref.ll)
    e_gp, e_gpk, k = param_errors(gp, ref, params)
    msg = f"  {label} {prec}: ll {ll:.15g} ref {ref.ll:.15g} | err ll {e_ll:.2e} gp {e_gp:.2e} gpk {e_gpk:.2e} (k={k})"
    out = {"ll": e_ll, "gp": e_gp, "gpk": e_gpk}
    if ref.gx is not None and gx is not None:
        rows = gx if ref.rows is None else gx[ref.rows]
        e_gx = rel_norm(rows, ref.gx)
        e_row, row, own = row_errors(rows, ref)
        msg += f" gx {e_gx:.2e} worst row {row}: {e_row:.2e} of its scale ({own:.2e} of its norm)"
        out.update(gx=e_gx, row=e_row)
    say(msg)
    for key, v in out.items():
        assert v <= tol[key], f"{label} {prec}: {key} error {v:.3e} above {tol[key]:.0e}"
    return out
