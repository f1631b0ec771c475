"""The autograd adjoint: gradcheck at small N, central finite differences on
the D = 6 influenza-like workload (N = 20,000), and the oracle's analytic
gradient."""
import numpy as np
import pytest
import torch

import oracle
from paper_2010_02994_amd import workloads as W
from paper_2010_02994_amd.autograd import hawkes_loglik
from tests.gpu_util import say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("d", [1, 2, 3])
def test_gradcheck_fp64(d):
    w = W.random_case(200 + d, 40, d, ties=1, t_span=3.0)
    x = torch.tensor(w.x, device=DEV, requires_grad=True)
    p = torch.tensor(w.params, dtype=torch.float64, requires_grad=True)
    t = torch.tensor(w.t, device=DEV)
    say(f"case gradcheck d={d}")
    assert torch.autograd.gradcheck(lambda a, b: hawkes_loglik(a, b, t, "fp64"), (x, p), eps=1e-6, atol=1e-6,
                                    rtol=1e-5, nondet_tol=0.0)


def test_backward_scales_and_refuses_double_backward():
    w = W.random_case(210, 100, 2, t_span=4.0)
    x = torch.tensor(w.x, device=DEV, requires_grad=True)
    p = torch.tensor(w.params, dtype=torch.float64, requires_grad=True)
    t = torch.tensor(w.t, device=DEV)
    say("case backward scaling")
    (2.5 * hawkes_loglik(x, p, t, "fp64")).backward()
    st, ll, gx, gp = oracle.loglik_grad(w.x, w.t, w.params)
    np.testing.assert_allclose(x.grad.cpu().numpy(), 2.5 * gx, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(p.grad.numpy(), 2.5 * gp, rtol=1e-10, atol=1e-12)
    x2 = torch.tensor(w.x, device=DEV, requires_grad=True)
    ll2 = hawkes_loglik(x2, p.detach(), t, "fp64")
    (g,) = torch.autograd.grad(ll2, x2, create_graph=True)
    with pytest.raises(RuntimeError):
        g.sum().backward()


def test_float32_inputs_return_float32_gradients():
    w = W.random_case(220, 300, 2, t_span=6.0)
    x = torch.tensor(w.x, device=DEV, dtype=torch.float32, requires_grad=True)
    p = torch.tensor(w.params, dtype=torch.float32, requires_grad=True)
    t = torch.tensor(w.t, device=DEV)
    say("case float32 inputs")
    hawkes_loglik(x, p, t, "mixed").backward()
    assert x.grad.dtype == torch.float32 and p.grad.dtype == torch.float32
    st, ll, gx, gp = oracle.loglik_grad(x.detach().double().cpu().numpy(), w.t, p.detach().double().numpy())
    assert np.linalg.norm(x.grad.double().cpu().numpy() - gx) <= 1e-4 * np.linalg.norm(gx)


@pytest.fixture(scope="module")
def c3():
    w = W.config3()
    rng = np.random.default_rng(1003)
    coords = [(int(i), int(k)) for i, k in zip(rng.integers(0, w.n, 50), rng.integers(0, w.d, 50))]
    st, ll, gx, gp = oracle.loglik_grad(w.x, w.t, w.params, threads=True)
    return w, coords, gx, gp


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_config3_finite_differences_and_oracle(c3, prec):
    """Central differences (step 1e-6) of the FP64 path's log-likelihood on 50
    seeded coordinates and all six parameters, against the autograd gradient of
    each precision; and the autograd gradient against the oracle's analytic one."""
    w, coords, gx_ref, gp_ref = c3
    t = torch.tensor(w.t, device=DEV)
    x = torch.tensor(w.x, device=DEV, requires_grad=True)
    p = torch.tensor(w.params, dtype=torch.float64, requires_grad=True)
    say(f"case config3 autograd prec={prec}")
    hawkes_loglik(x, p, t, prec).backward()
    gx = x.grad.cpu().numpy()
    gp = p.grad.numpy()

    def f64(xx, pp):
        with torch.no_grad():
            return float(hawkes_loglik(xx, pp, t, "fp64"))

    h = 1e-6
    fd_x, ad_x = [], []
    for (i, k) in coords:
        xp = x.detach().clone(); xp[i, k] += h
        xm = x.detach().clone(); xm[i, k] -= h
        fd_x.append((f64(xp, p.detach()) - f64(xm, p.detach())) / (2 * h))
        ad_x.append(gx[i, k])
    fd_p = []
    for k in range(6):
        hp = h * w.params[k]
        pp = p.detach().clone(); pp[k] += hp
        pm = p.detach().clone(); pm[k] -= hp
        fd_p.append((f64(x.detach(), pp) - f64(x.detach(), pm)) / (2 * hp))
    fd_x, ad_x, fd_p = np.array(fd_x), np.array(ad_x), np.array(fd_p)
    e_fd_x = np.linalg.norm(fd_x - ad_x) / np.linalg.norm(fd_x)
    e_fd_p = np.max(np.abs(w.params * (fd_p - gp))) / max(np.linalg.norm(w.params * gp), w.n)
    e_or_x = np.linalg.norm(gx - gx_ref) / np.linalg.norm(gx_ref)
    e_or_p = np.max(np.abs(w.params * (gp - gp_ref))) / max(np.linalg.norm(w.params * gp_ref), w.n)
    say(f"  {prec}: FD vs autograd x {e_fd_x:.2e} params {e_fd_p:.2e}; oracle vs autograd x {e_or_x:.2e} "
        f"params {e_or_p:.2e}")
    tol_fd = 1e-5 if prec == "fp64" else 1e-4
    tol_or = 1e-10 if prec == "fp64" else 1e-4
    assert e_fd_x <= tol_fd and e_fd_p <= tol_fd
    assert e_or_x <= tol_or and e_or_p <= tol_or


def test_bmds_gradcheck_and_joint_backward():
    """The MDS adjoint: torch.autograd.gradcheck in x and sigma (float64, small
    N), and the influenza model's joint log density hawkes + mds backpropagates
    the sum of the two library gradients."""
    from paper_2010_02994_amd import api
    from paper_2010_02994_amd.autograd import bmds_loglik
    c = W.bmds_case(230, 24, 3, missing=0.2)
    x = torch.tensor(c.x, device=DEV, requires_grad=True)
    s = torch.tensor(c.sigma, dtype=torch.float64, device=DEV, requires_grad=True)
    dl = torch.tensor(c.delta, device=DEV)
    say("case bmds gradcheck")
    assert torch.autograd.gradcheck(lambda xx, ss: bmds_loglik(xx, ss, dl, "fp64"), (x, s), eps=1e-6, atol=1e-6,
                                    rtol=1e-5)
    w, cf = W.flu_case(seed=231, n=400, d=6, groups=10, years=2.0)
    say("case joint hawkes + mds backward")
    for prec in ("fp64", "mixed"):
        xj = torch.tensor(w.x, device=DEV, requires_grad=True)
        t = torch.tensor(w.t, device=DEV)
        dj = torch.tensor(cf.delta, device=DEV)
        sj = torch.tensor(cf.sigma, dtype=torch.float64, device=DEV)
        p = torch.tensor(w.params, dtype=torch.float64)
        (hawkes_loglik(xj, p, t, prec) + bmds_loglik(xj, sj, dj, prec)).backward()
        _, gh, _ = api.grad(xj.detach(), t, w.params, prec=prec)
        _, gb = api.bmds(xj.detach(), dj, cf.sigma, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(xj.grad, gh + gb), prec
