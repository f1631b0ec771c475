"""GPU parity: the HIP library through the C ABI against the CPU oracle.

Every case compares the log-likelihood, every location-gradient row (with the
worst row against its own cancellation scale) and each parameter-gradient
component against its cancellation scale; metrics and tolerances are those of
tests/gpu_util.py (float64 1e-10; mixed 1e-5 / 1e-4 as the precision contract
states, 3e-4 per row and per component)."""
import math

import numpy as np
import pytest

import oracle
from paper_2010_02994_amd import workloads as W
from tests.gpu_util import check, oracle_ref, run_gpu, say

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "mixed"]


SMALL = [(1, 2, 1, 0), (2, 3, 2, 0), (3, 17, 2, 1), (4, 63, 3, 0), (5, 64, 2, 2), (6, 65, 1, 0), (7, 257, 6, 3),
         (8, 511, 2, 0), (9, 512, 2, 0), (10, 513, 8, 2), (11, 1000, 2, 4), (12, 1537, 3, 0), (13, 700, 5, 1),
         (14, 129, 4, 0), (15, 300, 7, 0)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("seed,n,d,ties", SMALL)
def test_random_cases(prec, seed, n, d, ties):
    w = W.random_case(seed, n, d, ties=ties, t_span=max(3.0, n / 40))
    say(f"case seed={seed} n={n} d={d} ties={ties} prec={prec}")
    ref = oracle_ref(w.x, w.t, w.params)
    check(prec, run_gpu(w.x, w.t, w.params, prec), ref, w.params, label=w.name)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("which", ["theta0", "mu_tiny"])
def test_single_component(prec, which):
    """theta = 0 (background only) and mu0 = 1e-9 (excitation dominates)."""
    w = W.random_case(21, 300, 2, ties=2, t_span=6.0)
    p = w.params.copy()
    if which == "theta0":
        p[3] = 0.0
    else:
        p[0] = 1e-9
    say(f"case single-component {which} prec={prec}")
    check(prec, run_gpu(w.x, w.t, p, prec), oracle_ref(w.x, w.t, p), p, label=which)


@pytest.mark.parametrize("prec", PRECS)
def test_mu_zero_is_zero_rate(prec):
    """mu0 = 0: the earliest event has no earlier partner, so its rate is 0."""
    w = W.random_case(22, 200, 2, t_span=6.0)
    p = w.params.copy()
    p[0] = 0.0
    st, ll, _, _ = oracle.loglik_grad(w.x, w.t, p)
    assert st == oracle.ZERORATE and ll == -math.inf
    say(f"case mu0=0 prec={prec}")
    ll_gpu, gx, gp = run_gpu(w.x, w.t, p, prec)
    assert ll_gpu == -math.inf and np.all(np.isnan(gx)) and np.all(np.isnan(gp))


@pytest.mark.parametrize("prec", PRECS)
def test_config0(prec):
    w = W.config0()
    say(f"case {w.name} prec={prec}")
    check(prec, run_gpu(w.x, w.t, w.params, prec), oracle_ref(w.x, w.t, w.params), w.params, label=w.name)


@pytest.fixture(scope="module")
def c1():
    return W.config1(snapshots=3)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("snap", [0, 3])
def test_config1_snapshots(c1, prec, snap):
    x = c1.x if snap == 0 else c1.snapshots[snap - 1]
    say(f"case {c1.name} snapshot={snap} prec={prec}")
    check(prec, run_gpu(x, c1.t, c1.params, prec), oracle_ref(x, c1.t, c1.params), c1.params,
          label=f"{c1.name}/s{snap}")


@pytest.mark.parametrize("prec", PRECS)
def test_config3_d6(prec):
    w = W.config3()
    say(f"case {w.name} prec={prec}")
    check(prec, run_gpu(w.x, w.t, w.params, prec), oracle_ref(w.x, w.t, w.params), w.params, label=w.name)


@pytest.fixture(scope="module")
def c2_ref():
    """The oracle at N = 50,000 (threaded): log-likelihood, parameter gradient
    with its cancellation scales, every location-gradient row with its scale,
    and the log-domain rates (for the fix-up diagnostics)."""
    w = W.config2()
    say(f"oracle {w.name} (threaded, every row) ...")
    ref = oracle_ref(w.x, w.t, w.params)
    log_lam, max_log_term = oracle.log_rates(w.x, w.t, w.params)
    return w, ref, log_lam, max_log_term


@pytest.mark.parametrize("prec", PRECS)
def test_config2_full_size(c2_ref, prec):
    """N = 50,000: the log-likelihood, the parameter gradient and all 50,000 x 2
    location-gradient entries against the oracle, with the worst row reported."""
    w, ref, _, _ = c2_ref
    say(f"case {w.name} prec={prec}")
    ll, gx, gp = run_gpu(w.x, w.t, w.params, prec)
    check(prec, (ll, gx, gp), ref, w.params, label=w.name)
    # translation invariance holds at any size: sum of gradients vanishes
    scale = np.abs(gx).sum(0)
    assert np.all(np.abs(gx.sum(0)) <= (1e-12 if prec == "fp64" else 1e-6) * scale)


@pytest.mark.parametrize("prec", PRECS)
def test_config2_fixup_rows(c2_ref, prec):
    """The rows the float64 fix-up recomputes at N = 50,000 are those the
    oracle's exact log-rates put below the scaled window: every row more than
    one binade below the threshold is flagged, none more than one above it.
    Mixed precision must flag some rows here (the workload has isolated events
    whose every pair term underflows float32 without the shift), and the rows
    with every term below the float32 range come out within tolerance (the
    full-size check covers every row)."""
    import torch
    from paper_2010_02994_amd import api
    w, ref, log_lam, max_log_term = c2_ref
    x = torch.tensor(w.x, device="cuda:0")
    t = torch.tensor(w.t, device="cuda:0")
    api.grad(x, t, w.params, prec=prec)
    info, flags = api.diagnostics(x, t, w.params, prec=prec)
    # log2 of lambda_n 2^S / (cmax 2^floor): negative means recompute
    margin = log_lam / math.log(2.0) + info["shift_log2"] - math.log2(info["cmax"]) - info["floor_log2"]
    must = margin < -1.0
    must_not = margin > 1.0
    below = max_log_term < oracle.FLT_MIN_LOG
    say(f"  {prec}: flagged {info['flagged_rows']} rows (S = {info['shift_log2']:.0f}, floor 2^{info['floor_log2']:.0f}); "
        f"oracle: {int(must.sum())} below the window by > 1 binade, {int((~must & ~must_not).sum())} within one binade; "
        f"{int(below.sum())} rows with every pair term below FLT_MIN, of which {int(flags[below].sum())} flagged")
    assert info["flagged_rows"] == int(flags.sum())
    assert np.all(flags[must] == 1) and np.all(flags[must_not] == 0)
    if prec == "mixed":
        assert info["flagged_rows"] > 0 and below.sum() > 0


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["c0", "c2", "c3"])
def test_no_gradient_variant(c2_ref, prec, case):
    """The rate pass without the location gradient (hawkes_loglik and
    hawkes_grad_async with grad_x = NULL; in mixed precision it accumulates the
    background moments itself) against the oracle: log-likelihood and each
    parameter-gradient component."""
    import torch
    from paper_2010_02994_amd import api
    if case == "c2":
        w, ref, _, _ = c2_ref
    else:
        w = W.config0() if case == "c0" else W.config3()
        ref = oracle_ref(w.x, w.t, w.params, want_gx=False)
    x = torch.tensor(w.x, device="cuda:0")
    t = torch.tensor(w.t, device="cuda:0")
    say(f"case no-gradient {w.name} prec={prec}")
    out8 = api.grad_async(x, t, w.params, prec=prec).cpu().numpy()
    assert out8[7] == 0
    check(prec, (out8[0], None, out8[1:7]), ref, w.params, label=f"{w.name} grad_x=NULL")
    ll = api.loglik(x, t, w.params, prec=prec)
    assert ll == out8[0]


def _isolated_case(lo=-700.0, hi=-630.0):
    """Moves event 5 about 28 bandwidths away (log rate near -300 relative to
    the pair weight: below the float32 window) and event 200 just far enough
    that its log rate falls between lo and hi (by default -700 to -630: below
    the float64 path's 2^-900 window, yet still positive in float64)."""
    w = W.random_case(31, 400, 2, t_span=10.0)
    p = np.array([0.5, 1.0, 1.0, 0.3, 1.0, 0.5])
    d = 2
    cmax = max(p[0] * (2 * np.pi) ** (-(d + 1) / 2) / p[1] ** d / p[2],
               p[3] * p[4] * (2 * np.pi) ** (-d / 2) / p[5] ** d)
    x = w.x.copy()
    x[5] += 20.0   # both coordinates: about 28 bandwidths away
    for off in np.arange(26.0, 34.0, 0.05):
        x[200] = w.x[200] - off
        lam, _ = oracle.rates(x, w.t, p)
        rel = np.log(lam[200] / cmax) if lam[200] > 0 else -np.inf
        if lo < rel < hi:
            return x, w.t, p
    raise AssertionError("could not place the isolated event")


@pytest.mark.parametrize("prec", PRECS)
def test_isolated_events_fixup(prec):
    """Rows far below the float32 window (and one below the float64 window) are
    recomputed exactly by the fix-up kernels."""
    x, t, p = _isolated_case()
    lam, _ = oracle.rates(x, t, p)
    say(f"case isolated prec={prec} min log lam {np.log(lam).min():.1f}")
    check(prec, run_gpu(x, t, p, prec), oracle_ref(x, t, p), p, label="isolated")


@pytest.mark.parametrize("prec", PRECS)
def test_isolated_event_subnormal_rate(prec):
    """An event whose rate is a float64 subnormal (about 1e-308), so every
    pair term it gets lies in the range where exp rounds into subnormals."""
    x, t, p = _isolated_case(-744.0, -600.0)
    # bisect the offset of event 200 (its rate falls as it moves away) to a
    # rate of 1e-308: subnormal, while 1/rate still fits in float64
    x0 = x[200] + 0.0
    lo, hi = -3.0, 3.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        x[200] = x0 - mid
        lam, _ = oracle.rates(x, t, p)
        lo, hi = (mid, hi) if lam[200] > 1e-308 else (lo, mid)
    x[200] = x0 - lo
    lam, _ = oracle.rates(x, t, p)
    st, ll_ref, gx_ref, gp_ref = oracle.loglik_grad(x, t, p, threads=True)
    assert st == 0 and np.all(np.isfinite(gp_ref)) and np.all(np.isfinite(gx_ref))
    say(f"case subnormal rate prec={prec} min rate {lam.min():.3e}")
    assert 1.0 / np.finfo(np.float64).max < lam.min() < np.finfo(np.float64).tiny
    check(prec, run_gpu(x, t, p, prec), oracle_ref(x, t, p), p, label="subnormal rate")


@pytest.mark.parametrize("prec", PRECS)
def test_translation_offset_mixed_stable(prec):
    """A large common offset must not degrade the result (float32 offsets are
    taken from the data center)."""
    w = W.random_case(41, 1000, 2, t_span=20.0)
    ref = oracle.loglik_grad(w.x, w.t, w.params, threads=True, want_grad_x=False)[1]
    say(f"case offset prec={prec}")
    check(prec, run_gpu(w.x + 5.0e4, w.t + 1.0e4, w.params, prec), oracle_ref(w.x + 5.0e4, w.t + 1.0e4, w.params),
          w.params, label="offset")
    # the oracle itself: a 5e4 offset costs ~1e-11 relative through float64
    # rounding of the shifted coordinates, so translation holds to 1e-9 here
    assert ref == pytest.approx(oracle.loglik_grad(w.x + 5.0e4, w.t, w.params, want_grad_x=False)[1], rel=1e-9)


@pytest.mark.parametrize("prec", PRECS)
def test_long_work_items_dense_cluster(prec):
    """Every tile of a band in one work item (HAWKES_TILES_PER_ITEM = 94 at
    N = 6,000, items of up to 6,016 columns) on a dense cluster whose pair
    terms all sit near their largest value (locations within ~1e-3 of the
    spatial bandwidths, times within half the temporal one): each item's row
    sums collect up to 6,000 near-maximal terms, which the float32
    micro-partials (at most 32 terms) and the float64 accumulators must carry
    without overflow."""
    import os
    w0 = W.random_case(41, 6000, 2, t_span=0.5)
    params = np.array([0.5, 1.0, 1.0, 0.5, 1.0, 0.5])
    x = np.ascontiguousarray(1e-3 * w0.x)
    say(f"case long work items, dense cluster n=6000 L=94 prec={prec}")
    ref = oracle_ref(x, w0.t, params)
    old = os.environ.get("HAWKES_TILES_PER_ITEM")
    os.environ["HAWKES_TILES_PER_ITEM"] = "94"
    try:
        got = run_gpu(x, w0.t, params, prec)
    finally:
        if old is None:
            os.environ.pop("HAWKES_TILES_PER_ITEM", None)
        else:
            os.environ["HAWKES_TILES_PER_ITEM"] = old
    assert np.isfinite(got[0])
    check(prec, got, ref, params, label="dense_cluster_n6000_L94")


@pytest.mark.parametrize("prec", PRECS)
def test_all_tied_is_zero_rate(prec):
    x = np.random.default_rng(1).standard_normal((70, 2))
    t = np.full(70, 1.5)
    say(f"case all-tied prec={prec}")
    ll, gx, gp = run_gpu(x, t, [0.5, 1, 1, 0.3, 1, 0.5], prec)
    assert ll == -math.inf and np.all(np.isnan(gx)) and np.all(np.isnan(gp))


@pytest.mark.parametrize("prec", PRECS)
def test_deterministic_bitwise(prec):
    w = W.random_case(51, 3000, 2, ties=3, t_span=60.0)
    say(f"case determinism prec={prec}")
    a = run_gpu(w.x, w.t, w.params, prec)
    b = run_gpu(w.x, w.t, w.params, prec)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_invalid_inputs_return_status_and_leave_outputs():
    import torch
    from paper_2010_02994_amd import _lib, api
    rng = np.random.default_rng(3)
    x = torch.tensor(rng.standard_normal((100, 2)), device="cuda:0")
    t_ok = np.sort(rng.uniform(0, 5, 100))
    p = [0.5, 1, 1, 0.3, 1, 0.5]
    say("case invalid inputs")
    for bad_t, bad_x in ((t_ok[::-1].copy(), None), (t_ok - 1.0, None), (t_ok, "nan")):
        tt = torch.tensor(bad_t, device="cuda:0")
        xx = x.clone()
        if bad_x == "nan":
            xx[7, 1] = float("nan")
        sentinel = torch.full_like(xx, 123.0)
        with pytest.raises(_lib.HawkesError) as e:
            api.grad(xx, tt, p, prec="mixed", out=sentinel)
        assert e.value.status == _lib.EDATA
        torch.cuda.synchronize()
        assert bool((sentinel == 123.0).all())
    for badp in ([0.5, -1, 1, 0.3, 1, 0.5], [0, 1, 1, 0, 1, 0.5], [0.5, 1, 1, 0.3, float("inf"), 0.5]):
        with pytest.raises(_lib.HawkesError) as e:
            api.grad(x, torch.tensor(t_ok, device="cuda:0"), badp)
        assert e.value.status == _lib.EPARAM


def _grad_in_order(x_np, t_np, params, prec):
    """The same evaluation through hawkes_grad_timed, which runs every stage in
    order on the caller's stream (no side stream)."""
    import ctypes
    import torch
    from paper_2010_02994_amd import _lib, api
    x = torch.tensor(np.ascontiguousarray(x_np), device="cuda:0")
    t = torch.tensor(np.ascontiguousarray(t_np), device="cuda:0")
    n, d = x.shape
    ws = api.workspace(n, d, prec, x.device)
    gx = torch.empty_like(x)
    ll = ctypes.c_double()
    gp = (ctypes.c_double * 6)()
    stage = (ctypes.c_float * 12)()
    ps = api.params_struct(params)
    st = _lib.lib().hawkes_grad_timed(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), api._prec(prec),
                                      ws.data_ptr(), ws.numel(), api._stream_ptr(x.device), ctypes.byref(ll),
                                      gx.data_ptr(), gp, stage)
    assert st == 0, _lib.strerror(st)
    return ll.value, gx.cpu().numpy(), np.array(gp[:])


@pytest.mark.parametrize("prec", PRECS)
def test_side_stream_matches_in_order(prec):
    """hawkes_grad runs the fix-ups and finalize on a side stream during pass 2;
    the results equal the all-in-order run bit for bit (flagged rows present)."""
    x, t, p = _isolated_case()
    say(f"case side-stream vs in-order prec={prec}")
    a = run_gpu(x, t, p, prec)
    b = _grad_in_order(x, t, p, prec)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("prec", PRECS)
def test_sync_scalars_equal_async_out8(prec):
    """hawkes_grad delivers its scalars through a pinned buffer that its last
    kernel writes: they equal hawkes_grad_async's device out8 bit for bit, the
    host outputs may be NULL, and a following call with other data gets its
    own values."""
    import ctypes
    import torch
    from paper_2010_02994_amd import _lib, api
    L = _lib.lib()
    for w in (W.random_case(81, 3000, 2, ties=2, t_span=30.0), W.random_case(82, 700, 3)):
        say(f"case sync scalars vs async out8 n={w.n} prec={prec}")
        x = torch.tensor(w.x, device="cuda:0")
        t = torch.tensor(w.t, device="cuda:0")
        n, d = x.shape
        ws = api.workspace(n, d, prec, x.device)
        ps = api.params_struct(w.params)
        s = api._stream_ptr(x.device)
        gx_a = torch.empty_like(x)
        out8 = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda:0")
        st = L.hawkes_grad_async(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), api._prec(prec), ws.data_ptr(),
                                 ws.numel(), s, out8.data_ptr(), gx_a.data_ptr())
        assert st == 0, _lib.strerror(st)
        torch.cuda.synchronize()
        o = out8.cpu().numpy()
        ll = ctypes.c_double(float("nan"))
        gp = (ctypes.c_double * 6)()
        gx = torch.empty_like(x)
        st = L.hawkes_grad(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), api._prec(prec), ws.data_ptr(),
                           ws.numel(), s, ctypes.byref(ll), gx.data_ptr(), gp)
        assert st == 0, _lib.strerror(st)
        assert o[7] == 0.0 and ll.value == o[0] and np.array_equal(np.array(gp[:]), o[1:7])
        gx2 = torch.empty_like(x)
        st = L.hawkes_grad(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), api._prec(prec), ws.data_ptr(),
                           ws.numel(), s, None, gx2.data_ptr(), None)
        assert st == 0, _lib.strerror(st)
        torch.cuda.synchronize()
        assert torch.equal(gx, gx_a) and torch.equal(gx2, gx_a)


@pytest.mark.parametrize("prec", PRECS)
def test_concurrent_callers_on_own_streams(prec):
    """Four host threads, each on its own stream with its own data, call
    hawkes_grad three times; every result equals a lone call's bit for bit."""
    import threading
    import torch
    from paper_2010_02994_amd import api
    cases = [W.random_case(60 + k, n, 2, ties=2, t_span=40.0) for k, n in enumerate((1500, 4000, 9000, 600))]
    dev_in = [(torch.tensor(w.x, device="cuda:0"), torch.tensor(w.t, device="cuda:0")) for w in cases]
    alone = [run_gpu(w.x, w.t, w.params, prec) for w in cases]
    torch.cuda.synchronize()
    out = [[None] * 3 for _ in cases]
    errs = []

    def worker(k):
        try:
            s = torch.cuda.Stream(device="cuda:0")
            with torch.cuda.stream(s):
                for r in range(3):
                    ll, gx, gp = api.grad(dev_in[k][0], dev_in[k][1], cases[k].params, prec=prec)
                    out[k][r] = (ll, gx.cpu().numpy(), gp)
        except Exception as e:   # surfaced below
            errs.append(repr(e))

    say(f"case concurrent callers prec={prec}")
    th = [threading.Thread(target=worker, args=(k,)) for k in range(len(cases))]
    for h in th:
        h.start()
    for h in th:
        h.join(timeout=120)
    assert not errs, errs
    for k, w in enumerate(cases):
        for r in range(3):
            a, b = out[k][r], alone[k]
            assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]), (k, r)


@pytest.mark.parametrize("prec", PRECS)
def test_exact_culling_is_bitwise_identical(prec):
    """A window much longer than the temporal scales: most column tiles lie so
    far in the past that both pair terms are exactly zero and are skipped; every
    output is bit for bit the one of the all-pairs run, and matches the oracle."""
    w = W.random_case(71, 6000, 2, ties=3, t_span=20000.0)
    say(f"case exact culling prec={prec} params={np.round(w.params, 3).tolist()}")
    a = run_gpu(w.x, w.t, w.params, prec)
    b = run_gpu(w.x, w.t, w.params, prec + "+cull")
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    check(prec, b, oracle_ref(w.x, w.t, w.params), w.params, label="culled")


@pytest.fixture(scope="module")
def big_case():
    """The wildfire-like generator at N = 300,000 (six times the benchmark
    size; 9e10 ordered pairs): too large for the oracle, so it is checked
    through identities that hold at any size and against a float64 oracle
    evaluation of the compensator alone."""
    w = W.config2(n=300000)
    p = w.params
    T = w.t.max()
    from scipy import stats
    comp = (p[0] * (stats.norm.cdf((T - w.t) / p[2]) - stats.norm.cdf(-w.t / p[2]))
            + p[3] * (1 - np.exp(-p[4] * (T - w.t))))
    return w, math.fsum(comp)


@pytest.mark.parametrize("prec", PRECS)
def test_largest_size_identities(big_case, prec):
    """At N = 300,000: the location gradient sums to zero (translation), the
    weights' Euler identity mu0 d/dmu0 + theta d/dtheta = N - sum Lambda_n holds,
    and the two precisions agree."""
    w, sum_comp = big_case
    say(f"case N=300000 identities prec={prec}")
    ll, gx, gp = run_gpu(w.x, w.t, w.params, prec)
    assert np.all(np.isfinite(gx)) and math.isfinite(ll)
    tol = 1e-10 if prec == "fp64" else 1e-5
    scale = np.abs(gx).sum(0)
    assert np.all(np.abs(gx.sum(0)) <= (1e-11 if prec == "fp64" else 1e-6) * scale)
    euler = w.params[0] * gp[0] + w.params[3] * gp[3]
    say(f"  euler {euler:.10g} vs {w.n - sum_comp:.10g}")
    assert abs(euler - (w.n - sum_comp)) <= tol * w.n
    if prec == "mixed":
        ll64, gx64, gp64 = run_gpu(w.x, w.t, w.params, "fp64")
        assert abs(ll - ll64) <= 1e-5 * abs(ll64)
        assert np.linalg.norm(gx - gx64) <= 1e-4 * np.linalg.norm(gx64)


def test_fp64_pair_exp_accuracy():
    """Two events: each per-event term is one pair term (an exp times a
    constant), so the float64 path's exp is checked directly against the
    oracle's over exponents from 0 to about -580.  The bound allows a few
    units in the last place for exp itself plus the rounding of the exponent
    (|z| units of 2^-53), which both sides form in their own order."""
    import torch
    from paper_2010_02994_amd import api
    p = np.array([0.5, 1.0, 1.0, 0.3, 1.0, 0.5])
    t = np.array([0.0, 0.5])
    worst, worst_ulp = 0.0, 0.0
    for s in np.concatenate([[1e-9, 1e-3, 0.1], np.linspace(0.5, 17.0, 34)]):
        x = np.array([[0.0], [s]])
        ref = oracle.event_terms(x, t, p)
        terms, _ = api.event_terms(torch.tensor(x, device="cuda:0"), torch.tensor(t, device="cuda:0"), p,
                                   prec="fp64")
        got = terms.cpu().numpy()
        z_bg = 0.5 * s * s + 0.5 * 0.25          # alpha r^2 + beta dt^2
        z_se = 1.0 * 0.5 + 2.0 * s * s           # omega dt + gamma r^2
        for (row, col), z in (((0, 0), z_bg), ((1, 0), z_bg), ((1, 1), z_se)):
            rel = abs(got[row, col] - ref[row, col]) / ref[row, col]
            worst = max(worst, rel / (8.0 + 2.0 * z))
            worst_ulp = max(worst_ulp, rel / 2.0 ** -53)
            assert rel <= (8.0 + 2.0 * z) * 2.0 ** -53, (s, row, col, rel)
        assert got[0, 1] == 0.0
    say(f"  fp64 exp: worst error {worst:.4f} of the bound, {worst_ulp:.1f} units of 2^-53")
