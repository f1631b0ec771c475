"""Pins for the CPU oracle: each test checks it against something other than
itself (a 50-digit evaluation from the rate functions, numerical quadrature,
library densities, algebraic invariants, finite differences)."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2010_02994_amd import workloads as W
from tests import mp_reference as R


def _case(seed, n, d, ties=0, params=None, scale=1.0, t_span=5.0):
    return W.random_case(seed, n, d, ties=ties, params=params, scale=scale, t_span=t_span)


# ---------------------------------------------------------------- rates ----

@pytest.mark.parametrize("seed,n,d", [(1, 2, 1), (2, 5, 2), (3, 8, 2), (4, 6, 3), (5, 7, 1)])
def test_rates_match_rate_functions_mpmath(seed, n, d):
    """lambda_n equals mu(x_n,t_n) + xi(x_n,t_n) of Sec. 2.1 evaluated at 50 digits."""
    w = _case(seed, n, d, t_span=3.0)
    lam, _ = oracle.rates(w.x, w.t, w.params)
    ref = R.rates_at_events(w.x.tolist(), w.t.tolist(), w.params.tolist())
    for a, b in zip(lam, ref):
        assert abs(a - float(b)) <= 1e-14 * abs(float(b))


@pytest.mark.parametrize("seed", [11, 12])
def test_rates_with_ties_match_rate_functions(seed):
    """Simultaneous events: background excluded, no excitation either way."""
    w = _case(seed, 8, 2, ties=3, t_span=2.0)
    assert len(np.unique(w.t)) < len(w.t)
    lam, _ = oracle.rates(w.x, w.t, w.params)
    ref = R.rates_at_events(w.x.tolist(), w.t.tolist(), w.params.tolist())
    for a, b in zip(lam, ref):
        assert abs(a - float(b)) <= 1e-14 * abs(float(b))


@pytest.mark.parametrize("d", [1, 2, 3])
def test_theta_zero_is_leave_one_out_kde(d):
    """theta = 0: lambda_n is mu0 times a leave-one-out Gaussian space-time KDE
    (scipy multivariate normal density), ties excluded."""
    w = _case(20 + d, 9, d, ties=2, t_span=2.0)
    p = w.params.copy()
    p[3] = 0.0
    lam, _ = oracle.rates(w.x, w.t, p)
    cov = np.diag([p[1] ** 2] * d + [p[2] ** 2])
    for i in range(w.n):
        s = 0.0
        for j in range(w.n):
            if j != i and w.t[j] != w.t[i]:
                s += stats.multivariate_normal.pdf(np.r_[w.x[i] - w.x[j], w.t[i] - w.t[j]], mean=np.zeros(d + 1), cov=cov)
        assert lam[i] == pytest.approx(p[0] * s, rel=1e-13)


@pytest.mark.parametrize("d", [1, 2, 6])
def test_mu_zero_is_exponential_gaussian_excitation(d):
    """mu0 = 0: lambda_n = theta omega sum_{t_n'<t_n} exp(-omega dt) N(dx; 0, h^2 I)."""
    w = _case(30 + d, 9, d, ties=2, t_span=2.0)
    p = w.params.copy()
    p[0] = 0.0
    lam, _ = oracle.rates(w.x, w.t, p)
    for i in range(w.n):
        s = 0.0
        for j in range(w.n):
            if w.t[j] < w.t[i]:
                s += math.exp(-p[4] * (w.t[i] - w.t[j])) * stats.multivariate_normal.pdf(
                    w.x[i] - w.x[j], mean=np.zeros(d), cov=p[5] ** 2 * np.eye(d))
        assert lam[i] == pytest.approx(p[3] * p[4] * s, rel=1e-13, abs=1e-300)


# ---------------------------------------------------------- compensator ----

def _space_time_quadrature(x, t, p, d):
    """Numerical integral of lambda(x, t) over R^D x [0, t_N]: composite
    Gauss-Legendre in every coordinate, time panels split at event times."""
    mu0, tx, tt, th, om, h = p
    lo = x.min() - 12 * max(tx, h)
    hi = x.max() + 12 * max(tx, h)
    bw = min(tx, h)
    npan = int(math.ceil((hi - lo) / (0.5 * bw)))
    g, gw = np.polynomial.legendre.leggauss(10)
    edges = np.linspace(lo, hi, npan + 1)
    xs = ((edges[:-1, None] + edges[1:, None]) / 2 + (edges[1:, None] - edges[:-1, None]) / 2 * g[None, :]).ravel()
    ws = ((edges[1:, None] - edges[:-1, None]) / 2 * gw[None, :]).ravel()
    grids = np.meshgrid(*([xs] * d), indexing="ij")
    pts = np.stack([gi.ravel() for gi in grids], axis=1)
    wsp = np.ones(1)
    for _ in range(d):
        wsp = np.multiply.outer(wsp, ws).ravel()

    def spatial_integral(tq):
        lamv = np.zeros(pts.shape[0])
        for n in range(len(t)):
            dx2 = ((pts - x[n]) ** 2).sum(1)
            # background rate mu(x,t) (t is never an event time at a Gauss node)
            lamv += mu0 / (tx ** d * tt) * (2 * np.pi) ** (-d / 2) * np.exp(-dx2 / (2 * tx * tx)) * \
                stats.norm.pdf((tq - t[n]) / tt)
            if t[n] < tq:
                lamv += th * om / h ** d * np.exp(-om * (tq - t[n])) * (2 * np.pi) ** (-d / 2) * \
                    np.exp(-dx2 / (2 * h * h))
        return float(wsp @ lamv)

    T = t.max()
    cuts = np.unique(np.r_[0.0, t[(t > 0) & (t < T)], T])
    total = 0.0
    gt, gtw = np.polynomial.legendre.leggauss(16)
    for a, b in zip(cuts[:-1], cuts[1:]):
        m = max(1, int(math.ceil((b - a) / (0.5 * min(tt, 1.0 / om)))))
        for k in range(m):
            aa, bb = a + (b - a) * k / m, a + (b - a) * (k + 1) / m
            for node, wt in zip(gt, gtw):
                total += (bb - aa) / 2 * wt * spatial_integral((aa + bb) / 2 + (bb - aa) / 2 * node)
    return total


@pytest.mark.parametrize("seed,n,d", [(41, 4, 1), (42, 5, 1), (43, 3, 2)])
def test_compensator_matches_space_time_quadrature(seed, n, d):
    """The closed-form Lambda(t_N) equals the numerical integral of the intensity
    over R^D x [0, t_N] (Sec. 2.1)."""
    p = np.array([0.7, 1.0, 0.8, 0.4, 1.3, 0.6])
    w = _case(seed, n, d, params=p, t_span=2.0, scale=0.5)
    st, ll, _, _ = oracle.loglik_grad(w.x, w.t, w.params, want_grad_x=False)
    lam, _ = oracle.rates(w.x, w.t, w.params)
    comp_oracle = float(np.sum(np.log(lam)) - ll)
    comp_num = _space_time_quadrature(w.x, w.t, w.params, d)
    assert comp_oracle == pytest.approx(comp_num, rel=1e-9)


@pytest.mark.parametrize("seed,n,d", [(51, 2, 1), (52, 5, 2), (53, 8, 3), (54, 7, 2)])
def test_loglik_matches_mpmath_rate_functions(seed, n, d):
    """ell from the oracle vs 50-digit log-rates minus a time quadrature of the
    spatially integrated rate."""
    w = _case(seed, n, d, ties=1 if n > 4 else 0, t_span=3.0)
    st, ll, _, _ = oracle.loglik_grad(w.x, w.t, w.params, want_grad_x=False)
    ref = float(R.loglik(w.x.tolist(), w.t.tolist(), w.params.tolist()))
    assert st == 0
    assert ll == pytest.approx(ref, rel=1e-13, abs=1e-12)


def test_two_events_closed_form():
    """N = 2 written out by hand: ell = log mu_12 + log(mu_21 + xi_21) - Lambda_1 - Lambda_2."""
    x = np.array([[0.3, -0.2], [0.1, 0.4]])
    t = np.array([0.5, 1.7])
    p = np.array([0.6, 0.9, 1.4, 0.5, 0.8, 0.7])
    mu0, tx, tt, th, om, h = p
    dx = x[1] - x[0]
    dt = t[1] - t[0]
    mu12 = mu0 * stats.multivariate_normal.pdf(np.r_[dx, dt], cov=np.diag([tx * tx, tx * tx, tt * tt]))
    xi21 = th * om * math.exp(-om * dt) * stats.multivariate_normal.pdf(dx, cov=h * h * np.eye(2))
    T = t[1]
    lam_c = [mu0 * (stats.norm.cdf((T - tn) / tt) - stats.norm.cdf(-tn / tt)) + th * (1 - math.exp(-om * (T - tn)))
             for tn in t]
    ref = math.log(mu12) + math.log(mu12 + xi21) - sum(lam_c)
    st, ll, _, _ = oracle.loglik_grad(x, t, p)
    assert ll == pytest.approx(ref, rel=1e-14)


# ------------------------------------------------------------ invariants ----

@pytest.mark.parametrize("d", [1, 2, 3])
def test_translation_and_permutation_invariance(d):
    w = _case(60 + d, 40, d, t_span=4.0)
    _, ll, _, _ = oracle.loglik_grad(w.x, w.t, w.params, want_grad_x=False)
    _, ll2, _, _ = oracle.loglik_grad(w.x + np.arange(1, d + 1) * 37.25, w.t, w.params, want_grad_x=False)
    perm = np.random.default_rng(d).permutation(w.n)
    _, ll3, _, _ = oracle.loglik_grad(w.x[perm], w.t[perm], w.params, want_grad_x=False)
    assert ll2 == pytest.approx(ll, rel=1e-12)
    assert ll3 == pytest.approx(ll, rel=1e-12)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_unit_scaling_identities(d):
    """Rescaling space by s (with both spatial bandwidths) shifts ell by -N D log s;
    rescaling time by s (tau_t -> s tau_t, omega -> omega/s) shifts it by -N log s."""
    w = _case(70 + d, 30, d, t_span=4.0)
    _, ll, _, _ = oracle.loglik_grad(w.x, w.t, w.params, want_grad_x=False)
    s = 3.7
    p = w.params.copy()
    p[1] *= s
    p[5] *= s
    _, lls, _, _ = oracle.loglik_grad(w.x * s, w.t, p, want_grad_x=False)
    assert lls == pytest.approx(ll - w.n * d * math.log(s), rel=1e-12)
    q = w.params.copy()
    q[2] *= s
    q[4] /= s
    _, llt, _, _ = oracle.loglik_grad(w.x, w.t * s, q, want_grad_x=False)
    assert llt == pytest.approx(ll - w.n * math.log(s), rel=1e-12)


def test_tie_removes_exactly_that_pair():
    """Moving an event onto another's time removes both pair terms between them,
    which equals the untied rates minus those two terms."""
    w = _case(80, 6, 2, t_span=3.0)
    t2 = w.t.copy()
    t2[3] = t2[2]
    lam_tie, _ = oracle.rates(w.x, t2, w.params)
    ref = R.rates_at_events(w.x.tolist(), t2.tolist(), w.params.tolist())
    for a, b in zip(lam_tie, ref):
        assert a == pytest.approx(float(b), rel=1e-14)
    # the tied pair contributes nothing to either event
    X = w.x.tolist()
    sub = [k for k in range(6) if k != 3]
    lam2_wo3 = R.background_rate(X[2], t2[2], [X[k] for k in sub], [t2[k] for k in sub], w.params.tolist()) + \
        R.excitation_rate(X[2], t2[2], [X[k] for k in sub], [t2[k] for k in sub], w.params.tolist())
    assert lam_tie[2] == pytest.approx(float(lam2_wo3), rel=1e-14)


# --------------------------------------------------------------- gradient ----

def _fd(f, v, i, step):
    a = v.copy()
    b = v.copy()
    a.flat[i] += step
    b.flat[i] -= step
    return (f(a) - f(b)) / (2 * step)


@pytest.mark.parametrize("seed,n,d", [(91, 12, 1), (92, 15, 2), (93, 10, 3), (94, 9, 6)])
def test_location_gradient_matches_central_differences(seed, n, d):
    w = _case(seed, n, d, ties=1, t_span=3.0)
    st, ll, gx, gp = oracle.loglik_grad(w.x, w.t, w.params)
    f = lambda xx: oracle.loglik_grad(xx, w.t, w.params, want_grad_x=False)[1]
    fd = np.array([_fd(f, w.x, i, 1e-6) for i in range(w.x.size)]).reshape(w.x.shape)
    assert np.linalg.norm(fd - gx) <= 1e-6 * np.linalg.norm(gx)


@pytest.mark.parametrize("seed,n,d", [(101, 12, 1), (102, 15, 2), (103, 10, 3)])
def test_parameter_gradient_matches_central_differences(seed, n, d):
    w = _case(seed, n, d, ties=1, t_span=3.0)
    st, ll, gx, gp = oracle.loglik_grad(w.x, w.t, w.params)
    f = lambda pp: oracle.loglik_grad(w.x, w.t, pp, want_grad_x=False)[1]
    for k in range(6):
        step = 1e-6 * w.params[k]
        fd = _fd(f, w.params, k, step)
        assert fd == pytest.approx(gp[k], rel=1e-6, abs=1e-7 * np.abs(gp).max())


def test_gradient_mpmath_derivative_tiny():
    """A coordinate and a parameter derivative against mpmath numerical
    differentiation of the 50-digit reference log-likelihood."""
    w = _case(111, 5, 2, t_span=2.0)
    st, ll, gx, gp = oracle.loglik_grad(w.x, w.t, w.params)
    X = w.x.tolist()

    def f_x(v):
        XX = [row[:] for row in X]
        XX[2][1] = v
        return R.loglik(XX, w.t.tolist(), w.params.tolist())

    def f_p(v):
        pp = w.params.tolist()
        pp[4] = v
        return R.loglik(X, w.t.tolist(), pp)

    assert gx[2, 1] == pytest.approx(float(mp.diff(f_x, mp.mpf(X[2][1]))), rel=1e-12)
    assert gp[4] == pytest.approx(float(mp.diff(f_p, mp.mpf(w.params[4]))), rel=1e-12)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_gradient_identities(d):
    """Sum of location gradients is zero (translation invariance); the spatial
    Euler identity sum_n x_n.g_n + tau_x dl/dtau_x + h dl/dh = -N D; the weight
    identity mu0 dl/dmu0 + theta dl/dtheta = N - sum_n Lambda_n."""
    w = _case(120 + d, 25, d, ties=2, t_span=4.0)
    st, ll, gx, gp = oracle.loglik_grad(w.x, w.t, w.params)
    lam, _ = oracle.rates(w.x, w.t, w.params)
    scale = np.abs(gx).sum()
    assert np.all(np.abs(gx.sum(0)) <= 1e-12 * scale)
    euler = float((w.x * gx).sum() + w.params[1] * gp[1] + w.params[5] * gp[5])
    assert euler == pytest.approx(-w.n * d, rel=1e-10)
    comp = float(np.log(lam).sum() - ll)
    assert w.params[0] * gp[0] + w.params[3] * gp[3] == pytest.approx(w.n - comp, rel=1e-10)


def test_zero_rate_is_flagged():
    """One isolated first event with mu0 = 0 has lambda = 0: ell = -inf."""
    x = np.array([[0.0, 0.0], [1.0, 1.0]])
    t = np.array([0.0, 1.0])
    p = np.array([0.0, 1.0, 1.0, 0.5, 1.0, 1.0])
    st, ll, gx, gp = oracle.loglik_grad(x, t, p)
    assert st == oracle.ZERORATE and ll == -math.inf


@pytest.mark.parametrize("seed,n,d", [(1, 2, 1), (4, 6, 3)])
def test_rate_rows_match_rate_functions_mpmath(seed, n, d):
    """rate_rows: the rates of listed events (in any order) equal mu + xi of
    Sec. 2.1 evaluated at 50 digits."""
    w = _case(seed, n, d, t_span=3.0)
    rows = np.arange(n)[::-1]
    lam, _ = oracle.rate_rows(w.x, w.t, w.params, rows)
    ref = R.rates_at_events(w.x.tolist(), w.t.tolist(), w.params.tolist())
    for r, a in zip(rows, lam):
        assert abs(a - float(ref[r])) <= 1e-14 * abs(float(ref[r]))


def test_rate_rows_equal_rates():
    """rate_rows gives the full evaluation's rates and row sums bit for bit
    (single-threaded and threaded builds), and refuses an index outside [0, n)."""
    w = _case(131, 60, 2, ties=3, t_span=3.0)
    lam, s6 = oracle.rates(w.x, w.t, w.params)
    rows = np.array([0, 59, 17, 17, 31])
    for threads in (False, True):
        l2, s2 = oracle.rate_rows(w.x, w.t, w.params, rows, threads=threads)
        assert np.array_equal(l2, lam[rows]) and np.array_equal(s2, s6[rows])
    with pytest.raises(ValueError):
        oracle.rate_rows(w.x, w.t, w.params, [60])


def test_grad_rows_equals_full_gradient():
    w = _case(130, 50, 2, ties=2, t_span=3.0)
    st, ll, gx, gp = oracle.loglik_grad(w.x, w.t, w.params)
    lam, _ = oracle.rates(w.x, w.t, w.params)
    rows = np.array([0, 7, 49, 13])
    assert np.array_equal(oracle.grad_rows(w.x, w.t, w.params, lam, rows), gx[rows])


def test_threaded_build_is_bitwise_identical():
    w = W.config0()
    a = oracle.loglik_grad(w.x[:300], w.t[:300], w.params)
    b = oracle.loglik_grad(w.x[:300], w.t[:300], w.params, threads=True)
    assert a[1] == b[1] and np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


# ------------------------------------- per-event terms and Metropolis moves ----

def _two_events():
    x = np.array([[0.3, -0.2], [0.1, 0.4]])
    t = np.array([0.5, 1.7])
    p = np.array([0.6, 0.9, 1.4, 0.5, 0.8, 0.7])
    return x, t, p


def _two_event_rates(x, t, p):
    """lambda_1, lambda_2 and their parts from scipy densities (Sec. 2.1)."""
    mu0, tx, tt, th, om, h = p
    dx = x[1] - x[0]
    dt = t[1] - t[0]
    a = stats.multivariate_normal.pdf(np.r_[dx, dt], cov=np.diag([tx * tx, tx * tx, tt * tt]))
    b2 = om * math.exp(-om * dt) * stats.multivariate_normal.pdf(dx, cov=h * h * np.eye(2))
    return a, b2


def test_event_terms_two_events_closed_form():
    """a_n, b_n, log lambda_n and the branching probability for N = 2."""
    x, t, p = _two_events()
    a, b2 = _two_event_rates(x, t, p)
    lam = [p[0] * a, p[0] * a + p[3] * b2]
    ref = np.array([[a, 0.0, math.log(lam[0]), 0.0], [a, b2, math.log(lam[1]), p[3] * b2 / lam[1]]])
    got = oracle.event_terms(x, t, p)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("d", [1, 2])
def test_branching_probability_limits(d):
    """theta = 0: no event has a parent; mu0 = 0: every event with an earlier
    event is a child with probability 1."""
    w = _case(70 + d, 30, d, ties=2, t_span=3.0)
    p = w.params.copy()
    p[3] = 0.0
    assert np.all(oracle.event_terms(w.x, w.t, p)[:, 3] == 0.0)
    p = w.params.copy()
    p[0] = 0.0
    got = oracle.event_terms(w.x, w.t, p)
    later = w.t > w.t.min()
    np.testing.assert_allclose(got[later, 3], 1.0, rtol=1e-15)


@pytest.mark.parametrize("seed,block", [(81, [4]), (82, [0, 9, 10]), (83, [3, 17, 18, 40])])
def test_mwg_delta_is_loglik_difference(seed, block):
    """The incremental change equals ell(after) - ell(before) of the full
    log-likelihood (whose compensator cancels), ties included."""
    w = _case(seed, 60, 2, ties=3, t_span=6.0)
    rng = np.random.default_rng(seed)
    xn = w.x[block] + 0.4 * rng.standard_normal((len(block), 2))
    delta, x1 = oracle.mwg_delta(w.x, w.t, w.params, block, xn)
    _, l0, _, _ = oracle.loglik_grad(w.x, w.t, w.params)
    _, l1, _, _ = oracle.loglik_grad(x1, w.t, w.params)
    assert delta == pytest.approx(l1 - l0, rel=1e-11, abs=1e-11 * abs(l0))


def test_mwg_delta_antisymmetric_and_additive():
    w = _case(84, 50, 2, ties=2, t_span=5.0)
    rng = np.random.default_rng(84)
    y = w.x.copy()
    y[[6, 11]] += 0.3 * rng.standard_normal((2, 2))
    z = y.copy()
    z[[11, 30]] += 0.3 * rng.standard_normal((2, 2))
    d_xy, _ = oracle.mwg_delta(w.x, w.t, w.params, [6, 11], y[[6, 11]])
    d_yx, _ = oracle.mwg_delta(y, w.t, w.params, [6, 11], w.x[[6, 11]])
    d_yz, _ = oracle.mwg_delta(y, w.t, w.params, [11, 30], z[[11, 30]])
    d_xz, _ = oracle.mwg_delta(w.x, w.t, w.params, [6, 11, 30], z[[6, 11, 30]])
    assert d_xy == pytest.approx(-d_yx, rel=1e-12, abs=1e-13)
    assert d_xy + d_yz == pytest.approx(d_xz, rel=1e-12, abs=1e-13)
    d0, _ = oracle.mwg_delta(w.x, w.t, w.params, [6], w.x[[6]])
    assert d0 == 0.0


def test_mwg_delta_two_events_closed_form():
    x, t, p = _two_events()
    x1 = x.copy()
    x1[1] = [0.9, -0.5]
    a0, b0 = _two_event_rates(x, t, p)
    a1, b1 = _two_event_rates(x1, t, p)
    ref = (math.log(p[0] * a1) + math.log(p[0] * a1 + p[3] * b1)
           - math.log(p[0] * a0) - math.log(p[0] * a0 + p[3] * b0))
    delta, _ = oracle.mwg_delta(x, t, p, [1], x1[[1]])
    assert delta == pytest.approx(ref, rel=1e-13)


def test_reweight_is_linear_in_the_weights():
    """ell at new (mu0, theta) rebuilt from the terms a_n, b_n and the
    compensator (scipy normal cdf) equals the full log-likelihood there."""
    w = _case(85, 40, 2, ties=2, t_span=4.0)
    terms = oracle.event_terms(w.x, w.t, w.params)
    p1 = w.params.copy()
    p1[0] *= 1.7
    p1[3] *= 0.4
    T = w.t.max()
    comp = (p1[0] * (stats.norm.cdf((T - w.t) / p1[2]) - stats.norm.cdf(-w.t / p1[2]))
            + p1[3] * (1 - np.exp(-p1[4] * (T - w.t))))
    ref = math.fsum(np.log(p1[0] * terms[:, 0] + p1[3] * terms[:, 1])) - math.fsum(comp)
    st, ll, gm, gt = oracle.loglik_reweight(w.x, w.t, p1)
    assert ll == pytest.approx(ref, rel=1e-12)
    lam = p1[0] * terms[:, 0] + p1[3] * terms[:, 1]
    cmu = stats.norm.cdf((T - w.t) / p1[2]) - stats.norm.cdf(-w.t / p1[2])
    assert gm == pytest.approx(math.fsum(terms[:, 0] / lam) - math.fsum(cmu), rel=1e-10)
    assert gt == pytest.approx(math.fsum(terms[:, 1] / lam) - math.fsum(1 - np.exp(-p1[4] * (T - w.t))), rel=1e-10)
