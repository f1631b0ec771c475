"""Seeded synthetic event sets shaped like the paper's three applications.

This module only draws random inputs: it holds none of the likelihood's
arithmetic, so both the HIP path and the CPU oracle can consume its output.

Parameter vectors use the order (mu, h, tau, theta, omega, xi), which maps to
the paper's Theta = (mu0, tau_x, tau_t, theta, omega, h) of Sec. 2.1:

    mu    = mu0    background weight
    h     = tau_x  background spatial bandwidth
    tau   = tau_t  background temporal bandwidth
    theta = theta  self-excitation weight
    omega = omega  self-excitation temporal decay rate
    xi    = h      self-excitation spatial bandwidth (the paper's h)

Workloads (one per configuration of the build's benchmark plan):

  0  N=1,000, D=2 exact locations in a 10 km box, one year (Sec. 2.1 model,
     small case the oracle finishes in well under a second).
  1  N=10,000, D=2 in a 20 km box; observed locations rounded to a 100 m grid
     and latent locations uniform in their cell (the square prior of
     Sec. 2.2.1, gunfire).  Twenty perturbed latent snapshots stand in for the
     positions an HMC trajectory visits.
  2  N=50,000, D=2 in a 500 km box over ten years; 30 % of the locations are
     latent uniform in discs of radius U(1,10) km (the disc prior of
     Sec. 2.2.2, wildfire).  Headline size.
  3  N=20,000 in D=6 latent coordinates (the BMDS "effective space" of
     Sec. 2.2.3, influenza).
  4  64 serving datasets, N log-uniform in [1e3, 1e5], coarsened like 1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PARAM_NAMES = ("mu", "h", "tau", "theta", "omega", "xi")


@dataclasses.dataclass
class Workload:
    name: str
    x: np.ndarray          # (N, D) float64, latent locations fed to the likelihood
    t: np.ndarray          # (N,) float64, sorted non-decreasing
    params: np.ndarray     # (6,) float64 in PARAM_NAMES order
    observed: np.ndarray | None = None   # (N, D) observed (coarsened) locations
    radius: np.ndarray | None = None     # (N,) disc radius, 0 where exact
    cell: float | None = None            # square cell side, when rounded to a grid
    snapshots: list | None = None        # extra latent configurations (list of (N, D))
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.t.shape[0])

    @property
    def d(self) -> int:
        return int(self.x.shape[1])


def _cluster_events(rng, n, frac_offspring, means, sd, box, t_max, off_sd, off_mean_dt, d=2):
    """Background points from an equal-weight Gaussian mixture clipped to the
    box, plus one generation of offspring displaced from a uniformly chosen
    background parent (a single-generation stand-in for the cluster process
    used in the paper's simulation study, App. C)."""
    n_off = int(round(frac_offspring * n))
    n_bg = n - n_off
    means = np.asarray(means, dtype=np.float64)
    comp = rng.integers(0, means.shape[0], size=n_bg)
    xb = means[comp] + sd * rng.standard_normal((n_bg, d))
    xb = np.clip(xb, 0.0, box)
    tb = rng.uniform(0.0, t_max, size=n_bg)
    parent = rng.integers(0, n_bg, size=n_off)
    xo = xb[parent] + off_sd * rng.standard_normal((n_off, d))
    to = tb[parent] + rng.exponential(off_mean_dt, size=n_off)
    x = np.concatenate([xb, xo], axis=0)
    t = np.concatenate([tb, to], axis=0)
    order = np.argsort(t, kind="stable")
    x = np.ascontiguousarray(x[order])
    t = np.ascontiguousarray(t[order])
    assert np.all(np.diff(t) > 0), "generator produced tied times"
    return x, t


def _coarsen_grid(rng, x, cell):
    """Round to a square grid and draw the latent location uniformly in its cell."""
    obs = np.round(x / cell) * cell
    lat = obs + rng.uniform(-0.5 * cell, 0.5 * cell, size=x.shape)
    return obs, lat


def _perturb_in_cells(rng, obs, lat, cell, step, count):
    """Seeded random-walk snapshots reflected at the cell walls (stand-ins for
    the positions an HMC trajectory visits; no gradient is involved)."""
    out = []
    cur = lat.copy()
    lo, hi = obs - 0.5 * cell, obs + 0.5 * cell
    for _ in range(count):
        cur = cur + step * rng.standard_normal(cur.shape)
        cur = np.where(cur < lo, 2 * lo - cur, cur)
        cur = np.where(cur > hi, 2 * hi - cur, cur)
        cur = np.clip(cur, lo, hi)
        out.append(np.ascontiguousarray(cur.copy()))
    return out


C0_PARAMS = np.array([0.5, 1.0, 10.0, 0.3, 0.5, 0.1])


def config0(seed: int = 1000) -> Workload:
    rng = np.random.default_rng(seed)
    x, t = _cluster_events(rng, 1000, 0.3, [(2, 2), (5, 7), (8, 3)], 0.8, 10.0, 365.0, 0.1, 2.0)
    return Workload("c0_n1000_d2_exact", x, t, C0_PARAMS.copy(), seed=seed)


def config1(seed: int = 1001, snapshots: int = 20) -> Workload:
    rng = np.random.default_rng(seed)
    x, t = _cluster_events(rng, 10000, 0.3, [(4, 4), (10, 14), (16, 6)], 1.6, 20.0, 365.0, 0.1, 2.0)
    obs, lat = _coarsen_grid(rng, x, 0.1)
    snaps = _perturb_in_cells(rng, obs, lat, 0.1, 0.002, snapshots)
    return Workload("c1_n10000_d2_grid100m", lat, t, C0_PARAMS.copy(), observed=obs, cell=0.1,
                    snapshots=snaps, seed=seed)


C2_PARAMS = np.array([0.5, 1.0, 10.0, 0.3, 0.1, 2.0])


def config2(seed: int = 1002, n: int = 50000, same_density: bool = False) -> Workload:
    """same_density: shrink the box (and the mixture) by sqrt(n / 50,000) so a
    smaller n keeps the 50,000-event workload's events per km^2 and day."""
    rng = np.random.default_rng(seed)
    s = float(np.sqrt(n / 50000.0)) if same_density else 1.0
    x, t = _cluster_events(rng, n, 0.2, [(100 * s, 100 * s), (250 * s, 350 * s), (400 * s, 150 * s)], 40.0 * s,
                           500.0 * s, 3650.0, 2.0, 10.0)
    obs = x.copy()
    n_disc = int(round(0.3 * n))
    idx = rng.choice(n, size=n_disc, replace=False)
    r = np.zeros(n)
    r[idx] = rng.uniform(1.0, 10.0, size=n_disc)
    u = rng.uniform(size=n_disc)
    v = rng.uniform(size=n_disc)
    lat = obs.copy()
    lat[idx, 0] += r[idx] * np.sqrt(u) * np.cos(2 * np.pi * v)
    lat[idx, 1] += r[idx] * np.sqrt(u) * np.sin(2 * np.pi * v)
    name = f"c2_n{n}_d2_disc" + (f"_box{500 * s:.0f}km" if same_density else "")
    return Workload(name, np.ascontiguousarray(lat), t, C2_PARAMS.copy(), observed=obs, radius=r, seed=seed)


C3_PARAMS = np.array([0.5, 1.0, 10.0, 0.3, 0.5, 0.05])


def config3(seed: int = 1003, n: int = 20000) -> Workload:
    rng = np.random.default_rng(seed)
    d = 6
    n_off = int(round(0.3 * n))
    n_bg = n - n_off
    xb = rng.standard_normal((n_bg, d))
    tb = rng.uniform(0.0, 730.0, size=n_bg)
    parent = rng.integers(0, n_bg, size=n_off)
    xo = xb[parent] + 0.05 * rng.standard_normal((n_off, d))
    to = tb[parent] + rng.exponential(2.0, size=n_off)
    x = np.concatenate([xb, xo])
    t = np.concatenate([tb, to])
    order = np.argsort(t, kind="stable")
    x, t = np.ascontiguousarray(x[order]), np.ascontiguousarray(t[order])
    assert np.all(np.diff(t) > 0)
    return Workload(f"c3_n{n}_d6_latent", x, t, C3_PARAMS.copy(), seed=seed)


def serving_sizes(count: int = 64, seed: int = 4, lo: float = 1e3, hi: float = 1e5) -> list[int]:
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(v))) for v in rng.uniform(math.log(lo), math.log(hi), size=count)]


def serving_dataset(k: int, n: int) -> Workload:
    rng = np.random.default_rng(40000 + k)
    x, t = _cluster_events(rng, n, 0.3, [(2, 2), (5, 7), (8, 3)], 0.8, 10.0, 365.0, 0.1, 2.0)
    obs, lat = _coarsen_grid(rng, x, 0.1)
    return Workload(f"c4_ds{k}_n{n}", lat, t, C0_PARAMS.copy(), observed=obs, cell=0.1, seed=40000 + k)


def serving_arrivals(rate: float, duration_s: float, chains: int = 64, seed: int = 4):
    """Open-loop Poisson arrival times (s) and the chain each request belongs to."""
    rng = np.random.default_rng(seed + 7)
    n = int(rng.poisson(rate * duration_s))
    times = np.sort(rng.uniform(0.0, duration_s, size=n))
    chain = rng.integers(0, chains, size=n)
    return times, chain


def random_case(seed: int, n: int, d: int, ties: int = 0, scale: float = 1.0,
                params: np.ndarray | None = None, t_span: float = 5.0) -> Workload:
    """Small random event set for parity and edge-case tests.  `ties` events
    copy the time of an earlier event (exact duplicates)."""
    rng = np.random.default_rng(seed)
    x = scale * rng.standard_normal((n, d))
    t = np.sort(rng.uniform(0.0, t_span, size=n))
    if ties and n >= 2:
        for _ in range(ties):
            i = int(rng.integers(1, n))
            t[i] = t[i - 1]
        t = np.sort(t)
    if params is None:
        params = np.array([rng.uniform(0.2, 1.0), rng.uniform(0.5, 2.0), rng.uniform(0.5, 3.0),
                           rng.uniform(0.1, 0.8), rng.uniform(0.3, 2.0), rng.uniform(0.2, 1.0)])
    return Workload(f"rand_s{seed}_n{n}_d{d}", np.ascontiguousarray(x), np.ascontiguousarray(t),
                    np.asarray(params, dtype=np.float64), seed=seed)


@dataclasses.dataclass
class BmdsCase:
    name: str
    x: np.ndarray        # (N, D) latent locations (the state a sampler moves)
    delta: np.ndarray    # (N, N) observed dissimilarities, symmetric, NaN where unobserved
    sigma: float
    seed: int


def bmds_case(seed: int, n: int, d: int, missing: float = 0.0, sigma: float = 0.3,
              groups: int = 0) -> BmdsCase:
    """Seeded dissimilarity data in the shape of the influenza application
    (Sec. 2.2.3): true positions z, observed delta = |z_n - z_n'| plus normal
    noise of sd sigma, folded to be positive; the latent x starts at z plus a
    perturbation.  With `groups` > 0 every event belongs to one of that many
    countries and delta is the distance between the country centres (the
    air-traffic matrix is country by country), with same-country pairs
    unobserved.  `missing` marks a further random fraction unobserved."""
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(seed)
    if groups > 0:
        centres = 2.0 * rng.standard_normal((groups, d))
        g = rng.integers(0, groups, size=n)
        z = centres[g] + 0.05 * rng.standard_normal((n, d))
        delta = cdist(centres, centres)[g][:, g]
    else:
        z = rng.standard_normal((n, d))
        delta = cdist(z, z)
    # symmetric folded noise: the strict lower triangle's draws mirrored
    noise = rng.standard_normal((n, n))
    noise *= sigma
    noise = np.tril(noise, -1)
    noise += noise.T
    delta += noise
    del noise
    np.abs(delta, out=delta)
    if groups > 0:
        delta[g[:, None] == g[None, :]] = np.nan
    if missing > 0:
        m = np.tril(rng.uniform(size=(n, n)) < missing, -1)
        m |= m.T
        delta[m] = np.nan
        del m
    np.fill_diagonal(delta, np.nan)
    x = z + 0.1 * rng.standard_normal((n, d))
    return BmdsCase(f"bmds_s{seed}_n{n}_d{d}", np.ascontiguousarray(x), np.ascontiguousarray(delta), float(sigma),
                    seed)


def bmds_case_device(seed: int, n: int, d: int, missing: float = 0.0, sigma: float = 0.3, groups: int = 0,
                     device="cuda:0"):
    """The recipe of `bmds_case` drawn with torch's seeded generator on
    `device`, for sizes whose N x N matrix is slow to build on the host.
    Returns (x, delta) as float64 device tensors and sigma."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    f64 = dict(generator=g, device=device, dtype=torch.float64)
    if groups > 0:
        centres = 2.0 * torch.randn((groups, d), **f64)
        grp = torch.randint(0, groups, (n,), generator=g, device=device)
        z = centres[grp] + 0.05 * torch.randn((n, d), **f64)
        delta = torch.cdist(centres, centres)[grp][:, grp].contiguous()
    else:
        z = torch.randn((n, d), **f64)
        delta = torch.cdist(z, z)
    noise = torch.randn((n, n), **f64).tril_(-1)
    delta.add_(sigma * (noise + noise.T)).abs_()
    del noise
    if groups > 0:
        delta[grp[:, None] == grp[None, :]] = float("nan")
    if missing > 0:
        m = (torch.rand((n, n), generator=g, device=device, dtype=torch.float64) < missing).tril_(-1)
        m |= m.T.clone()
        delta[m] = float("nan")
        del m
    delta.fill_diagonal_(float("nan"))
    x = z + 0.1 * torch.randn((n, d), **f64)
    return x.contiguous(), delta, float(sigma)


def flu_case(seed: int = 1004, n: int = 4733, d: int = 6, groups: int = 64, years: float = 12.0):
    """Joint Hawkes + Bayesian MDS workload in the shape of the influenza
    application (Sec. 4.3): `n` cases in `groups` countries over `years`
    years, latent locations in d dimensions with the country-by-country
    dissimilarities of `bmds_case`, case times uniform over the span (sorted,
    no ties).  Returns (Workload with the Hawkes inputs, BmdsCase)."""
    c = bmds_case(seed, n, d, groups=groups)
    return _flu_workload(seed, n, d, groups, years, c.x.copy()), c


def _flu_workload(seed, n, d, groups, years, x):
    rng = np.random.default_rng(seed + 1)
    t = np.sort(rng.uniform(0.0, 365.0 * years, size=n))
    assert np.all(np.diff(t) > 0)
    # (mu0, tau_x, tau_t, theta, omega, h): background kernel wide in the
    # latent space and half a year in time, self-excitation within a country
    params = np.array([0.5, 1.0, 180.0, 0.5, 0.01, 0.2])
    return Workload(f"flu_n{n}_d{d}_{groups}countries", np.ascontiguousarray(x), t, params, seed=seed)


def flu_case_device(seed: int = 1004, n: int = 4733, d: int = 6, groups: int = 64, years: float = 12.0,
                    device="cuda:0"):
    """`flu_case` with the dissimilarities drawn on the device
    (`bmds_case_device`).  Returns (Workload, delta tensor, sigma)."""
    x, delta, sigma = bmds_case_device(seed, n, d, groups=groups, device=device)
    return _flu_workload(seed, n, d, groups, years, x.cpu().numpy()), delta, sigma

