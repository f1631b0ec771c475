"""GPU parity of the per-event terms, the Metropolis-within-Gibbs location
step and the weight reweighting against the CPU oracle."""
import math

import numpy as np
import pytest

import oracle
from paper_2010_02994_amd import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "mixed"]


def _dev(a, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device="cuda:0", dtype=dtype)


def _check_terms(got, ref, prec, params, label="", mixed_tol=2e-5):
    """float64: each of a, b to 1e-10 of itself.  Mixed: a and b to mixed_tol
    of the rate they form (a part far below its row's rate lies under the
    float32 window and may read 0); log lambda and the probability absolutely."""
    tol = 1e-10 if prec == "fp64" else mixed_tol
    ok = np.isfinite(ref[:, 2])
    mu0, th = params[0], params[3]
    if prec == "fp64":
        sa, sb = np.abs(ref[:, 0]), np.abs(ref[:, 1])
        ca, cb = 1.0, 1.0
    else:
        lam = mu0 * ref[:, 0] + th * ref[:, 1]
        sa, sb = lam, lam
        ca, cb = mu0, th
    e_a = float(np.max(np.where(sa[ok] > 0, ca * np.abs(got[ok, 0] - ref[ok, 0]) / np.maximum(sa[ok], 1e-300),
                                np.abs(got[ok, 0]))))
    e_b = float(np.max(np.where(sb[ok] > 0, cb * np.abs(got[ok, 1] - ref[ok, 1]) / np.maximum(sb[ok], 1e-300),
                                np.abs(got[ok, 1]))))
    e_l = float(np.max(np.abs(got[ok, 2] - ref[ok, 2]) / np.maximum(1.0, np.abs(ref[ok, 2]))))
    e_p = float(np.max(np.abs(got[ok, 3] - ref[ok, 3])))
    say(f"  terms {label} {prec}: a {e_a:.2e} b {e_b:.2e} logl {e_l:.2e} p {e_p:.2e}")
    assert e_a <= tol and e_b <= tol and e_l <= tol and e_p <= tol


@pytest.mark.parametrize("prec", PRECS)
def test_event_terms_random(prec):
    from paper_2010_02994_amd import api
    w = W.random_case(90, 1500, 2, ties=3, t_span=30.0)
    say(f"case event-terms n=1500 prec={prec}")
    terms, ll = api.event_terms(_dev(w.x), _dev(w.t), w.params, prec=prec)
    ref = oracle.event_terms(w.x, w.t, w.params)
    _check_terms(terms.cpu().numpy(), ref, prec, w.params, "random")
    _, ll_ref, _, _ = oracle.loglik_grad(w.x, w.t, w.params, threads=True, want_grad_x=False)
    assert ll == pytest.approx(ll_ref, rel=1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", PRECS)
def test_event_terms_d6_and_isolated_rows(prec):
    """D = 6, and rows whose rate sits below the float32 window (recomputed by
    the fix-up kernels) still get exact terms."""
    from paper_2010_02994_amd import api
    w = W.random_case(91, 700, 6, t_span=20.0)
    x = w.x.copy()
    x[3] += 9.0
    say(f"case event-terms d=6 isolated prec={prec}")
    terms, _ = api.event_terms(_dev(x), _dev(w.t), w.params, prec=prec)
    _check_terms(terms.cpu().numpy(), oracle.event_terms(x, w.t, w.params), prec, w.params, "d6")


_n530 = {}


@pytest.mark.parametrize("prec", PRECS)
def test_event_terms_more_than_1024_bands(prec):
    """N = 530,000 (1,036 row bands of 512 events, so the set-up kernel lays
    out the work items in two rounds of 1,024 bands; the second round holds
    bands 11 down to 0): the per-event terms of about 200 events, from the
    first band to the last, against the oracle's rates of those events alone.
    The wildfire-like events span ~250 bandwidths, so in mixed precision a
    pair term carries a relative error up to ~1e-4 from the float32
    coordinates, and a rate, a weighted mean of its terms' errors, is held to
    the worst-row bar of 3e-4 of the gradient rows."""
    from paper_2010_02994_amd import api
    if not _n530:
        w = W.config2(n=530000)
        rng = np.random.default_rng(530)
        rows = np.unique(np.concatenate([[0, 1, 511, 512, 6143, 6144, w.n - 1], rng.integers(0, 6144, 20),
                                         rng.integers(0, w.n, 180)]))
        _n530.update(w=w, rows=rows, ref=oracle.event_terms(w.x, w.t, w.params, rows=rows))
    w, rows, ref = _n530["w"], _n530["rows"], _n530["ref"]
    say(f"case event-terms n={w.n} rows={len(rows)} prec={prec}")
    terms, _ = api.event_terms(_dev(w.x), _dev(w.t), w.params, prec=prec)
    _check_terms(terms.cpu().numpy()[rows], ref, prec, w.params, "n530000", mixed_tol=3e-4)


def _state(w, x=None):
    from paper_2010_02994_amd import api
    x = w.x if x is None else x
    xd, td = _dev(x), _dev(w.t)
    terms, _ = api.event_terms(xd, td, w.params, prec="fp64")
    return xd, td, terms


@pytest.mark.parametrize("block", [[7], [3, 4, 5], list(range(100, 1900, 90))])
def test_mwg_single_step_accept_and_reject(block):
    import torch
    from paper_2010_02994_amd import api
    w = W.random_case(92, 2000, 2, ties=4, t_span=40.0)
    rng = np.random.default_rng(92)
    xn = w.x[block] + 0.3 * rng.standard_normal((len(block), 2))
    ref_delta, x1 = oracle.mwg_delta(w.x, w.t, w.params, block, xn)
    say(f"case mwg block={len(block)}")
    # reject: threshold +inf leaves everything bitwise unchanged
    xd, td, terms = _state(w)
    x0, terms0 = xd.clone(), terms.clone()
    idx, xnd = _dev(np.array(block, dtype=np.int64)), _dev(xn)
    out = api.mwg_step(xd, td, w.params, terms, idx, xnd, _dev([math.inf]))
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    say(f"  delta {o[0]:.15g} ref {ref_delta:.15g}")
    assert o[2] == 0 and o[1] == 0
    assert abs(o[0] - ref_delta) <= 1e-10 + 1e-10 * abs(ref_delta)
    assert torch.equal(xd, x0) and torch.equal(terms, terms0)
    # accept: threshold -inf
    out = api.mwg_step(xd, td, w.params, terms, idx, xnd, _dev([-math.inf]))
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert o[1] == 1 and abs(o[0] - ref_delta) <= 1e-10 + 1e-10 * abs(ref_delta)
    assert np.array_equal(xd.cpu().numpy(), x1)
    _check_terms(terms.cpu().numpy(), oracle.event_terms(x1, w.t, w.params), "fp64", w.params, "after accept")


def test_mwg_cancelled_rate_is_recomputed_exactly():
    """A tight pair far from everything: moving one of them away leaves the
    other with a rate many orders of magnitude smaller, which the incremental
    update cannot resolve; the row is recomputed in full."""
    import torch
    from paper_2010_02994_amd import api
    w = W.random_case(93, 800, 2, t_span=30.0)
    x = w.x.copy()
    k = 400
    c = 18.0 * w.params[1]   # about 25 background bandwidths from the cloud
    x[k] = [c, c]
    x[k + 1] = [c + 0.05 * w.params[1], c + 0.02 * w.params[1]]
    xn = np.array([[-c, 0.9 * c]])
    ref_delta, x1 = oracle.mwg_delta(x, w.t, w.params, [k + 1], xn)
    lam_after, _ = oracle.rates(x1, w.t, w.params)
    lam_before, _ = oracle.rates(x, w.t, w.params)
    say(f"case mwg cancellation ref delta {ref_delta:.6g} rate of the partner {lam_before[k]:.3g} -> "
        f"{lam_after[k]:.3g}")
    assert np.isfinite(ref_delta) and lam_after[k] < 1e-30 * lam_before[k]
    xd, td, terms = _state(w, x)
    out = api.mwg_step(xd, td, w.params, terms, _dev(np.array([k + 1], dtype=np.int64)), _dev(xn),
                       _dev([-math.inf]))
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    say(f"  delta {o[0]:.15g}")
    assert o[1] == 1 and abs(o[0] - ref_delta) <= 1e-9 * abs(ref_delta)
    ref = oracle.event_terms(x1, w.t, w.params)
    got = terms.cpu().numpy()
    assert got[k, 0] == pytest.approx(ref[k, 0], rel=1e-10)
    assert got[k, 2] == pytest.approx(ref[k, 2], rel=1e-12)
    _check_terms(got, ref, "fp64", w.params, "cancellation")


def test_mwg_chain_matches_oracle_decisions():
    """A 60-step random-scan chain (uniform disc proposals around the observed
    location, uniform log thresholds), enqueued without host synchronization;
    every Delta ell and decision equals the oracle's, and the final cached
    terms equal a fresh evaluation."""
    import torch
    from paper_2010_02994_amd import api
    w = W.random_case(94, 600, 2, ties=2, t_span=25.0)
    rng = np.random.default_rng(94)
    steps, radius = 60, 0.4
    obs = w.x.copy()
    idx = rng.integers(0, w.n, size=steps)
    ang = rng.uniform(0, 2 * np.pi, steps)
    rad = radius * np.sqrt(rng.uniform(size=steps))
    xn = obs[idx] + np.c_[rad * np.cos(ang), rad * np.sin(ang)]
    thr = np.log(rng.uniform(size=steps))
    say("case mwg chain 60 steps")
    xd, td, terms = _state(w)
    idx_d, xn_d, thr_d = _dev(idx.astype(np.int64)), _dev(xn), _dev(thr)
    outs = torch.empty((steps, 3), dtype=torch.float64, device="cuda:0")
    for s in range(steps):
        api.mwg_step(xd, td, w.params, terms, idx_d[s:s + 1], xn_d[s:s + 1], thr_d[s:s + 1], out3=outs[s])
    torch.cuda.synchronize()
    got = outs.cpu().numpy()
    x = w.x.copy()
    acc = 0
    for s in range(steps):
        d_ref, x1 = oracle.mwg_delta(x, w.t, w.params, [idx[s]], xn[s:s + 1])
        assert abs(got[s, 0] - d_ref) <= 1e-9 + 1e-9 * abs(d_ref), (s, got[s, 0], d_ref)
        assert abs(d_ref - thr[s]) > 1e-6, "near-tie decision; pick another seed"
        take = d_ref > thr[s]
        assert got[s, 1] == (1.0 if take else 0.0), s
        if take:
            x = x1
            acc += 1
    say(f"  accepted {acc} of {steps}")
    assert 0 < acc < steps
    assert np.array_equal(xd.cpu().numpy(), x)
    _check_terms(terms.cpu().numpy(), oracle.event_terms(x, w.t, w.params), "fp64", w.params, "after chain")


def test_mwg_invalid_block_is_rejected_without_change():
    import torch
    from paper_2010_02994_amd import api
    w = W.random_case(95, 300, 2, t_span=10.0)
    xd, td, terms = _state(w)
    x0, terms0 = xd.clone(), terms.clone()
    say("case mwg invalid blocks")
    for bad in ([5, 5], [9, 2], [3, w.n + 7]):
        out = api.mwg_step(xd, td, w.params, terms, _dev(np.array(bad, dtype=np.int64)),
                           _dev(w.x[[0, 1]] + 0.1), _dev([-math.inf]))
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        assert np.isnan(o[0]) and o[1] == 0 and o[2] == -3, bad
    out = api.mwg_step(xd, td, w.params, terms, _dev(np.array([4], dtype=np.int64)), _dev([[np.nan, 0.0]]),
                       _dev([-math.inf]))
    torch.cuda.synchronize()
    assert out.cpu().numpy()[2] == -3
    assert torch.equal(xd, x0) and torch.equal(terms, terms0)


def test_loglik_reweight():
    import torch
    from paper_2010_02994_amd import api
    w = W.random_case(96, 1200, 2, ties=2, t_span=30.0)
    _, td, terms = _state(w)
    say("case reweight")
    for f_mu, f_th in ((1.0, 1.0), (1.6, 0.3), (0.2, 2.5)):
        p1 = w.params.copy()
        p1[0] *= f_mu
        p1[3] *= f_th
        out = api.loglik_reweight(td, 2, p1, terms)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        st, ll, gm, gt = oracle.loglik_reweight(w.x, w.t, p1)
        say(f"  ({f_mu}, {f_th}): ll {o[0]:.15g} ref {ll:.15g}")
        assert o[0] == pytest.approx(ll, rel=1e-12)
        assert abs(o[1] - gm) <= 1e-10 * max(abs(gm), w.n)
        assert abs(o[2] - gt) <= 1e-10 * max(abs(gt), w.n)


@pytest.mark.parametrize("n,block", [(2925, 64), (2925, 200), (6000, 64)])
def test_mwg_large_blocks_match_oracle(n, block):
    """Blocks of many moved events on the wildfire-like workload (latent disc
    locations, same events per km^2 and day as N = 50,000): Delta ell against
    the oracle, reject and accept, and the cached terms after accepting."""
    import torch
    from paper_2010_02994_amd import api
    w = W.config2(n=n, same_density=True)
    rng = np.random.default_rng(n + block)
    latent = np.flatnonzero(w.radius > 0)
    idx = np.sort(rng.choice(latent, size=block, replace=False))
    ang = rng.uniform(0, 2 * np.pi, block)
    rad = w.radius[idx] * np.sqrt(rng.uniform(size=block))
    xn = w.observed[idx] + np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=-1)
    ref_delta, x1 = oracle.mwg_delta(w.x, w.t, w.params, list(idx), xn)
    say(f"case mwg n={n} block={block}: ref delta {ref_delta:.10g}")
    xd, td, terms = _state(w)
    idx_d, xn_d = _dev(idx.astype(np.int64)), _dev(xn)
    out = api.mwg_step(xd, td, w.params, terms, idx_d, xn_d, _dev([math.inf]))
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    say(f"  gpu delta {o[0]:.10g} status {o[2]}")
    assert o[2] == 0 and o[1] == 0
    assert abs(o[0] - ref_delta) <= 1e-9 * max(1.0, abs(ref_delta))
    out = api.mwg_step(xd, td, w.params, terms, idx_d, xn_d, _dev([-math.inf]))
    torch.cuda.synchronize()
    assert out.cpu().numpy()[1] == 1
    assert np.array_equal(xd.cpu().numpy(), x1)
    _check_terms(terms.cpu().numpy(), oracle.event_terms(x1, w.t, w.params), "fp64", w.params, "large block")
