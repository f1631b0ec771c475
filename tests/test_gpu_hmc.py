"""GPU parity of the device-resident leapfrog trajectories (reflecting box and
disc walls) against the oracle's trajectories."""
import numpy as np
import pytest

import oracle
from oracle import hmc
from paper_2010_02994_amd import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device="cuda:0")


def _run(w, p0, eps, steps, prec, bound, b0, b1):
    import torch
    from paper_2010_02994_amd import api
    x, p, t = _dev(w.x), _dev(p0), _dev(w.t)
    kind = {hmc.NONE: None, hmc.BOX: "box", hmc.DISC: "disc"}[bound]
    g, out8 = api.leapfrog(x, p, t, w.params, eps, steps, prec=prec, bound=kind,
                           b0=_dev(b0) if b0 is not None else None, b1=_dev(b1) if b1 is not None else None)
    torch.cuda.synchronize()
    return x.cpu().numpy(), p.cpu().numpy(), g.cpu().numpy(), out8.cpu().numpy()


def _case(kind, d=2):
    if kind == "cells":
        # 100 m grid cells around the observed points, as in the gridded workload
        w = W.random_case(101, 1500, d, ties=2, scale=1.0, t_span=40.0)
        obs = np.round(w.x / 0.1) * 0.1
        return w, hmc.BOX, obs - 0.05, obs + 0.05
    w = W.random_case(102, 1500, d, ties=2, scale=1.0, t_span=40.0)
    rng = np.random.default_rng(102)
    r = np.where(rng.uniform(size=w.n) < 0.3, 0.0, rng.uniform(0.02, 0.2, w.n))
    ang = rng.standard_normal((w.n, d))
    ang /= np.linalg.norm(ang, axis=1, keepdims=True)
    centre = w.x - ang * (r * rng.uniform(0, 1, w.n))[:, None]
    return w, hmc.DISC, centre, r


@pytest.mark.parametrize("kind,d", [("cells", 2), ("discs", 2), ("discs", 3)])
def test_leapfrog_fp64_matches_oracle(kind, d):
    w, bound, b0, b1 = _case(kind, d)
    rng = np.random.default_rng(103)
    p0 = rng.standard_normal(w.x.shape)
    eps, steps = 0.004, 20
    say(f"case leapfrog fp64 {kind} d={d} n={w.n}")
    x, p, g, out8 = _run(w, p0, eps, steps, "fp64", bound, b0, b1)
    xr, pr, gr = hmc.leapfrog(w.x, p0, eps, steps, hmc.hawkes_grad_fn(w.t, w.params), bound, b0, b1)
    moved = np.linalg.norm(xr - w.x)
    flips = int(np.sum(np.sign(pr) != np.sign(p0)))
    e_x = np.linalg.norm(x - xr) / moved
    e_p = np.linalg.norm(p - pr) / np.linalg.norm(pr)
    e_g = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    say(f"  err x {e_x:.2e} p {e_p:.2e} grad {e_g:.2e} (momentum sign changes {flips})")
    assert out8[7] == 0
    assert flips > 0
    assert e_x <= 1e-9 and e_p <= 1e-9 and e_g <= 1e-9
    if bound == hmc.BOX:
        assert np.all(x >= b0) and np.all(x <= b1)
    else:
        assert np.all(np.linalg.norm(x - b0, axis=1) <= b1 * (1 + 1e-14) + 1e-300)


def test_leapfrog_mixed_unbounded_matches_oracle():
    w = W.random_case(104, 2000, 2, ties=2, t_span=40.0)
    rng = np.random.default_rng(104)
    p0 = rng.standard_normal(w.x.shape)
    eps, steps = 0.01, 20
    say("case leapfrog mixed unbounded")
    x, p, g, out8 = _run(w, p0, eps, steps, "mixed", hmc.NONE, None, None)
    xr, pr, gr = hmc.leapfrog(w.x, p0, eps, steps, hmc.hawkes_grad_fn(w.t, w.params))
    e_x = np.linalg.norm(x - xr) / np.linalg.norm(xr - w.x)
    e_dp = np.linalg.norm(p - pr) / np.linalg.norm(pr - p0)
    say(f"  err displacement {e_x:.2e} momentum change {e_dp:.2e}")
    assert out8[7] == 0 and e_x <= 1e-4 and e_dp <= 1e-4


def test_leapfrog_chained_trajectories():
    """Two 5-step trajectories, the second reusing the first's final gradient,
    equal one 10-step trajectory (the two half kicks at the seam add up to the
    interior kick)."""
    import torch
    from paper_2010_02994_amd import api
    w, bound, b0, b1 = _case("cells")
    rng = np.random.default_rng(105)
    p0 = rng.standard_normal(w.x.shape)
    say("case leapfrog chained")
    xa, pa, ga, _ = _run(w, p0, 0.004, 10, "fp64", bound, b0, b1)
    x, p, t = _dev(w.x), _dev(p0), _dev(w.t)
    g, _ = api.leapfrog(x, p, t, w.params, 0.004, 5, prec="fp64", bound="box", b0=_dev(b0), b1=_dev(b1))
    g, _ = api.leapfrog(x, p, t, w.params, 0.004, 5, prec="fp64", bound="box", b0=_dev(b0), b1=_dev(b1),
                        grad_x=g, have_grad=True)
    torch.cuda.synchronize()
    np.testing.assert_allclose(x.cpu().numpy(), xa, rtol=0, atol=1e-13)
    np.testing.assert_allclose(p.cpu().numpy(), pa, rtol=1e-12, atol=1e-12)
    assert np.array_equal(g.cpu().numpy(), ga) or np.allclose(g.cpu().numpy(), ga, rtol=1e-12)


def test_leapfrog_graph_replay_matches_eager():
    """A 5-step trajectory captured once in a HIP graph (through torch's
    graph capture; the library's side stream joins the capture through its
    events) and replayed three times, with eager work and synchronizations
    between the replays, gives bit for bit the states of three eager
    trajectories."""
    import torch
    from paper_2010_02994_amd import api
    w, bound, b0, b1 = _case("cells")
    rng = np.random.default_rng(106)
    p0 = rng.standard_normal(w.x.shape)
    t, lo, hi = _dev(w.t), _dev(b0), _dev(b1)
    say("case leapfrog graph replay")
    for prec in ("mixed", "fp64"):
        # eager reference: first gradient, then three chained 5-step trajectories
        x, p = _dev(w.x), _dev(p0)
        g, _ = api.leapfrog(x, p, t, w.params, 0.004, 1, prec=prec, bound="box", b0=lo, b1=hi)
        x0, p0d, g0 = x.clone(), p.clone(), g.clone()
        eager = []
        for _ in range(3):
            g, out8 = api.leapfrog(x, p, t, w.params, 0.004, 5, prec=prec, bound="box", b0=lo, b1=hi,
                                   grad_x=g, have_grad=True)
            torch.cuda.synchronize()
            eager.append((x.cpu().numpy(), p.cpu().numpy(), g.cpu().numpy(), out8.cpu().numpy()))
        # graph: capture one trajectory on the same state buffers
        xs, ps, gs = x0.clone(), p0d.clone(), g0.clone()
        out8g = torch.empty(8, dtype=torch.float64, device="cuda:0")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):   # warm the capture stream's workspace outside the capture
            api.leapfrog(xs.clone(), ps.clone(), t, w.params, 0.004, 1, prec=prec, bound="box", b0=lo, b1=hi,
                         grad_x=gs.clone(), have_grad=True, out8=out8g)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            api.leapfrog(xs, ps, t, w.params, 0.004, 5, prec=prec, bound="box", b0=lo, b1=hi,
                         grad_x=gs, have_grad=True, out8=out8g)
        xs.copy_(x0); ps.copy_(p0d); gs.copy_(g0)
        torch.cuda.synchronize()
        for k in range(3):
            graph.replay()
            torch.cuda.synchronize()
            got = (xs.cpu().numpy(), ps.cpu().numpy(), gs.cpu().numpy(), out8g.cpu().numpy())
            _ = (xs * 2).sum().item()   # unrelated eager work between replays
            for a, b in zip(got, eager[k]):
                assert np.array_equal(a, b), (prec, k)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_leapfrog_bmds_matches_oracle(prec):
    """The influenza model's joint trajectory (Hawkes + MDS potential, D = 6)
    against the oracle's leapfrog with the summed gradients."""
    import torch
    from paper_2010_02994_amd import api
    w, c = W.flu_case(seed=107, n=700, d=6, groups=16, years=4.0)
    rng = np.random.default_rng(107)
    p0 = rng.standard_normal(w.x.shape)
    eps, steps = 0.002, 10
    say(f"case leapfrog+bmds {prec} n={w.n} d=6")
    x, p, t, dl = _dev(w.x), _dev(p0), _dev(w.t), _dev(c.delta)
    g, out8, out4 = api.leapfrog_bmds(x, p, t, w.params, dl, c.sigma, eps, steps, prec=prec)
    torch.cuda.synchronize()
    x, p, g, out8, out4 = (v.cpu().numpy() for v in (x, p, g, out8, out4))
    xr, pr, gr = hmc.leapfrog(w.x, p0, eps, steps, hmc.joint_grad_fn(w.t, w.params, c.delta, c.sigma))
    e_x = np.linalg.norm(x - xr) / np.linalg.norm(xr - w.x)
    e_dp = np.linalg.norm(p - pr) / np.linalg.norm(pr - p0)
    e_g = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    say(f"  err displacement {e_x:.2e} momentum change {e_dp:.2e} grad {e_g:.2e}")
    assert out8[7] == 0 and out4[3] == 0
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert e_x <= tol and e_dp <= tol and e_g <= tol
    st, ll_b, _, M, _ = oracle.bmds(xr, c.delta, c.sigma)
    assert out4[2] == M
    assert abs(out4[0] - ll_b) <= (1e-10 if prec == "fp64" else 1e-5) * abs(ll_b)


def test_leapfrog_bmds_gradient_is_the_sum_of_the_single_calls():
    """At the trajectory's end, the returned gradient equals the Hawkes and
    MDS location gradients of the single entry points added (bitwise), and
    out8/out4 equal those calls' outputs."""
    import torch
    from paper_2010_02994_amd import api
    w, c = W.flu_case(seed=108, n=500, d=6, groups=12, years=3.0)
    rng = np.random.default_rng(108)
    say("case leapfrog+bmds gradient sum")
    for prec in ("mixed", "fp64"):
        x, p, t, dl = _dev(w.x), _dev(rng.standard_normal(w.x.shape)), _dev(w.t), _dev(c.delta)
        g, out8, out4 = api.leapfrog_bmds(x, p, t, w.params, dl, c.sigma, 0.002, 3, prec=prec)
        gh = torch.empty_like(x)
        o8 = api.grad_async(x, t, w.params, prec=prec, grad_x=gh)
        o4, gb = api.bmds(x, dl, c.sigma, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(g, gh + gb), prec
        assert torch.equal(out8, o8) and torch.equal(out4, o4), prec


def test_leapfrog_bmds_graph_replay_matches_eager():
    """The joint trajectory (its MDS pair pass on a side stream beside each
    Hawkes evaluation) captured once in a HIP graph and replayed three times,
    with eager work between the replays, equals three eager trajectories bit
    for bit."""
    import torch
    from paper_2010_02994_amd import api
    w, c = W.flu_case(seed=109, n=600, d=6, groups=12, years=3.0)
    rng = np.random.default_rng(109)
    p0 = rng.standard_normal(w.x.shape)
    t, dl = _dev(w.t), _dev(c.delta)
    say("case leapfrog+bmds graph replay")
    for prec in ("mixed", "fp64"):
        x, p = _dev(w.x), _dev(p0)
        g, _, _ = api.leapfrog_bmds(x, p, t, w.params, dl, c.sigma, 0.002, 1, prec=prec)
        x0, p0d, g0 = x.clone(), p.clone(), g.clone()
        eager = []
        for _ in range(3):
            g, o8, o4 = api.leapfrog_bmds(x, p, t, w.params, dl, c.sigma, 0.002, 4, prec=prec, grad_x=g,
                                          have_grad=True)
            torch.cuda.synchronize()
            eager.append(tuple(v.cpu().numpy() for v in (x, p, g, o8, o4)))
        xs, ps, gs = x0.clone(), p0d.clone(), g0.clone()
        o8g = torch.empty(8, dtype=torch.float64, device="cuda:0")
        o4g = torch.empty(4, dtype=torch.float64, device="cuda:0")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):   # warm the capture stream's workspaces outside the capture
            api.leapfrog_bmds(xs.clone(), ps.clone(), t, w.params, dl, c.sigma, 0.002, 1, prec=prec,
                              grad_x=gs.clone(), have_grad=True, out8=o8g, out4=o4g)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            api.leapfrog_bmds(xs, ps, t, w.params, dl, c.sigma, 0.002, 4, prec=prec, grad_x=gs, have_grad=True,
                              out8=o8g, out4=o4g)
        xs.copy_(x0); ps.copy_(p0d); gs.copy_(g0)
        torch.cuda.synchronize()
        for k in range(3):
            graph.replay()
            torch.cuda.synchronize()
            got = tuple(v.cpu().numpy() for v in (xs, ps, gs, o8g, o4g))
            _ = (xs * 2).sum().item()   # unrelated eager work between replays
            for a, b in zip(got, eager[k]):
                assert np.array_equal(a, b), (prec, k)
