"""Pins of the oracle's Bayesian MDS log-likelihood (Sec. 2.2.3, eq.
bmdsLikelihood) to scipy's truncated normal, finite differences and the
invariances of a likelihood of distances."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2010_02994_amd import workloads as W


def _full(ll_oracle, M):
    """The paper's density drops the (2 pi)^{-M/2}; add it back."""
    return ll_oracle - 0.5 * M * math.log(2 * math.pi)


@pytest.mark.parametrize("seed,n,d,missing", [(1, 2, 2, 0.0), (2, 7, 2, 0.0), (3, 9, 3, 0.3), (4, 6, 6, 0.0)])
def test_bmds_is_truncated_normal_density(seed, n, d, missing):
    c = W.bmds_case(seed, n, d, missing=missing)
    st, ll, _, M, _ = oracle.bmds(c.x, c.delta, c.sigma)
    assert st == 0
    ref, cnt = 0.0, 0
    for i in range(n):
        for j in range(i):
            v = c.delta[i, j]
            if np.isnan(v):
                continue
            dd = float(np.linalg.norm(c.x[i] - c.x[j]))
            ref += stats.truncnorm.logpdf(v, a=-dd / c.sigma, b=np.inf, loc=dd, scale=c.sigma)
            cnt += 1
    assert M == cnt
    assert _full(ll, M) == pytest.approx(ref, rel=1e-13, abs=1e-13)


def _fd(f, v, step):
    return (f(v + step) - f(v - step)) / (2 * step)


@pytest.mark.parametrize("seed,d", [(11, 2), (12, 6)])
def test_bmds_gradients_match_central_differences(seed, d):
    c = W.bmds_case(seed, 12, d, missing=0.2)
    st, ll, ds, M, gx = oracle.bmds(c.x, c.delta, c.sigma)
    for (i, k) in [(0, 0), (5, d - 1), (11, 1)]:
        def f(v, i=i, k=k):
            x = c.x.copy()
            x[i, k] = v
            return oracle.bmds(x, c.delta, c.sigma, want_grad_x=False)[1]
        assert gx[i, k] == pytest.approx(_fd(f, c.x[i, k], 1e-6), rel=1e-6, abs=1e-7)
    g = _fd(lambda s: oracle.bmds(c.x, c.delta, s, want_grad_x=False)[1], c.sigma, 1e-6)
    assert ds == pytest.approx(g, rel=1e-6)


@pytest.mark.parametrize("d", [2, 3])
def test_bmds_invariances(d):
    """A likelihood of distances: invariant under rigid motions (so the
    gradient sums to zero and sum_n x_n g_n^T is symmetric), and scaling
    x, delta and sigma by s subtracts M log s."""
    c = W.bmds_case(20 + d, 15, d, missing=0.1)
    st, ll, ds, M, gx = oracle.bmds(c.x, c.delta, c.sigma)
    rng = np.random.default_rng(d)
    q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    x2 = c.x @ q.T + rng.standard_normal(d)
    assert oracle.bmds(x2, c.delta, c.sigma)[1] == pytest.approx(ll, rel=1e-12)
    np.testing.assert_allclose(gx.sum(0), 0.0, atol=1e-11 * np.abs(gx).sum())
    A = c.x.T @ gx
    np.testing.assert_allclose(A - A.T, 0.0, atol=1e-11 * np.abs(A).sum())
    s = 3.7
    ll_s = oracle.bmds(s * c.x, s * c.delta, s * c.sigma)[1]
    assert ll_s == pytest.approx(ll - M * math.log(s), rel=1e-12)


def test_bmds_single_observed_pair_closed_form():
    """Every pair missing but one: ell = -log sigma - (delta - d)^2/(2 sigma^2) - log Phi(d/sigma)."""
    c = W.bmds_case(30, 6, 2, missing=0.0)
    delta = np.full_like(c.delta, np.nan)
    delta[4, 1] = 2.5
    st, ll, ds, M, gx = oracle.bmds(c.x, delta, c.sigma)
    dd = float(np.linalg.norm(c.x[4] - c.x[1]))
    ref = -math.log(c.sigma) - (2.5 - dd) ** 2 / (2 * c.sigma ** 2) - math.log(stats.norm.cdf(dd / c.sigma))
    assert M == 1 and ll == pytest.approx(ref, rel=1e-14)
    assert np.all(gx[[0, 2, 3, 5]] == 0.0)
    np.testing.assert_allclose(gx[4], -gx[1], rtol=1e-15)


def test_bmds_rejects_invalid_delta():
    c = W.bmds_case(31, 5, 2)
    bad = c.delta.copy()
    bad[3, 1] = -0.5
    assert oracle.bmds(c.x, bad, c.sigma)[0] == -1
    bad[3, 1] = np.inf
    assert oracle.bmds(c.x, bad, c.sigma)[0] == -1
