"""Leapfrog trajectories with reflecting walls, for checking the device
trajectories.

TEST INFRASTRUCTURE ONLY: used by tests/; the product path never imports it.

Written from the definitions (arXiv 2010.02994, Sec. 3: HMC with unit mass and
the leapfrog integrator; Sec. 2.2: each location confined to a box or a disc
around its observed position).  The potential is -ell, so a kick adds
eps * grad ell to the momentum.  A wall mirrors the motion: a box wall flips
the momentum component normal to it, a sphere (disc for d = 2) reflects the
momentum about the normal at the contact point.  Bounds with zero width (or
zero radius) pin the coordinate (location) and leave its momentum alone; a
flight meeting more than 64 sphere walls stops at the wall.
"""
from __future__ import annotations

import numpy as np

from . import bmds, loglik_grad

NONE, BOX, DISC = 0, 1, 2
MAX_BOUNCES = 64


def fly_box(x, p, lo, hi, eps):
    """Straight flight for time eps, mirrored wall by wall until inside."""
    x = np.asarray(x, dtype=np.float64)
    p = np.array(p, dtype=np.float64, copy=True)
    pinned = ~(hi > lo)
    xn = x + eps * p
    while True:
        over = (xn > hi) & ~pinned
        under = (xn < lo) & ~pinned
        if not (over.any() or under.any()):
            break
        xn = np.where(over, 2.0 * hi - xn, xn)
        p = np.where(over, -p, p)
        xn = np.where(under, 2.0 * lo - xn, xn)
        p = np.where(under, -p, p)
    return np.where(pinned, lo, xn), p


def fly_ball(x, p, c, r, eps):
    """Straight flight for time eps inside |x - c| <= r per row: the contact
    time is the positive root of |y + s p|^2 = r^2 (quadratic formula); at
    contact p <- p - 2 (p.n) n with n = y / |y|."""
    x = np.array(x, dtype=np.float64, copy=True)
    p = np.array(p, dtype=np.float64, copy=True)
    for i in range(x.shape[0]):
        if not r[i] > 0:
            x[i] = c[i]
            continue
        y = x[i] - c[i]
        v = p[i].copy()
        rem = eps
        for _ in range(MAX_BOUNCES):
            a = v @ v
            if a == 0.0:
                break
            b = 2.0 * (y @ v)
            cc = y @ y - r[i] ** 2
            s = (-b + np.sqrt(max(b * b - 4.0 * a * cc, 0.0))) / (2.0 * a)
            if s >= rem:
                y = y + rem * v
                rem = 0.0
                break
            y = y + s * v
            rem -= s
            nrm = y / np.linalg.norm(y)
            v = v - 2.0 * (v @ nrm) * nrm
        if np.linalg.norm(y) > r[i]:
            y = y * (r[i] / np.linalg.norm(y))
        x[i] = c[i] + y
        p[i] = v
    return x, p


def fly(x, p, eps, bound=NONE, b0=None, b1=None):
    if bound == BOX:
        return fly_box(x, p, b0, b1, eps)
    if bound == DISC:
        return fly_ball(x, p, b0, b1, eps)
    return x + eps * p, np.array(p, copy=True)


def hawkes_grad_fn(t, params):
    def g(x):
        st, _, gx, _ = loglik_grad(x, t, params, threads=True)
        return gx
    return g


def bmds_grad_fn(delta, sigma):
    """Location gradient of the Bayesian MDS log-likelihood (Sec. 2.2.3)."""
    def g(x):
        st, _, _, _, gx = bmds(x, delta, sigma)
        return gx
    return g


def joint_grad_fn(t, params, delta, sigma):
    """Gradient of the influenza model's log density over the locations
    (Sec. 3): the Hawkes log-likelihood plus the MDS log-likelihood."""
    gh, gb = hawkes_grad_fn(t, params), bmds_grad_fn(delta, sigma)
    return lambda x: gh(x) + gb(x)


def leapfrog(x, p, eps, steps, grad_fn, bound=NONE, b0=None, b1=None, g0=None):
    """steps leapfrog steps, each a kick of eps/2, a flight for time eps and a
    kick of eps/2.  Returns (x, p, gradient at the final x)."""
    x = np.array(x, dtype=np.float64, copy=True)
    p = np.array(p, dtype=np.float64, copy=True)
    g = grad_fn(x) if g0 is None else g0
    for _ in range(steps):
        p = p + 0.5 * eps * g
        x, p = fly(x, p, eps, bound, b0, b1)
        g = grad_fn(x)
        p = p + 0.5 * eps * g
    return x, p, g
