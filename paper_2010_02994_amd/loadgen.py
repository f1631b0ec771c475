"""Open-loop load generator for the serving benchmark (64 HMC chains over
datasets of uneven N, Poisson arrivals).  Each chain's latent locations take
small uniform steps reflected inside their 100 m cells (generated on the device
before the run), and each request asks the server for log-likelihood +
gradient at the chain's next step.  Latency runs from the scheduled arrival to
completion; the client is never allowed to hide queueing by submitting late
without counting it."""
from __future__ import annotations

import time

import numpy as np
import torch

from . import workloads
from .serve import Server


class Chains:
    def __init__(self, server: Server, count: int = 64, seed: int = 4, lo: float = 1e3, hi: float = 1e5,
                 device: str = "cuda:0"):
        self.sizes = workloads.serving_sizes(count, seed, lo, hi)
        self.dev = torch.device(device)
        self.ds, self.t, self.x, self.lo, self.hi, self.params = [], [], [], [], [], []
        for k, n in enumerate(self.sizes):
            w = workloads.serving_dataset(k, n)
            t = torch.tensor(w.t, device=self.dev)
            self.t.append(t)
            self.ds.append(server.register(t, w.d))
            self.x.append(torch.tensor(w.x, device=self.dev))
            self.lo.append(torch.tensor(w.observed - 0.5 * w.cell, device=self.dev))
            self.hi.append(torch.tensor(w.observed + 0.5 * w.cell, device=self.dev))
            self.params.append(w.params)
        self.gen = torch.Generator(device=self.dev)
        self.gen.manual_seed(seed)

    def step(self, k: int, scale: float = 0.002) -> torch.Tensor:
        """New latent positions of chain k (a fresh tensor: an in-flight
        request keeps its own copy)."""
        x = self.x[k]
        u = torch.rand(x.shape, device=self.dev, dtype=x.dtype, generator=self.gen)
        y = x + scale * (2.0 * u - 1.0)
        y = torch.where(y < self.lo[k], 2 * self.lo[k] - y, y)
        y = torch.where(y > self.hi[k], 2 * self.hi[k] - y, y)
        y = torch.minimum(torch.maximum(y, self.lo[k]), self.hi[k])
        self.x[k] = y
        return y

    def prepare(self, ring: int = 8, want_grad: bool = True):
        """Pre-generate, on the device, `ring` consecutive random-walk steps of
        every chain and as many output buffers, so that submitting a request
        costs the client no device work; request j of chain k uses step
        j mod ring (the chain cycles through its walk)."""
        self.ring = ring
        self.pos = [[self.step(k) for _ in range(ring)] for k in range(len(self.sizes))]
        self.out = [[torch.empty_like(self.x[k]) if want_grad else None for _ in range(ring)]
                    for k in range(len(self.sizes))]
        self.used = [0] * len(self.sizes)
        torch.cuda.synchronize(self.dev)


def run(server: Server, chains: Chains, rate: float, n_requests: int, prec: str = "mixed",
        warmup_s: float = 5.0, seed: int = 4, want_grad: bool = True, timeout_s: float = 300.0) -> dict:
    """Open-loop Poisson arrivals at `rate` per second, each picking a chain
    uniformly; requests arriving in the first warmup_s seconds run but are not
    measured, then n_requests are.  Latency = completion - scheduled arrival
    (client lag and queueing included).  Also reported: the server's queue wait
    (admission - submission), launch wait (start - admission) and service time
    (completion - start), the achieved submission rate, and the throughput
    (all completions, warm-up ones included, between the first measured
    arrival and the last measured completion, over that time), which at an
    offered rate above capacity is the capacity."""
    if not hasattr(chains, "pos"):
        chains.prepare(want_grad=want_grad)
    rng = np.random.default_rng(seed + 11)
    n_warm = int(np.ceil(rate * warmup_s))
    total = n_warm + n_requests
    gaps = rng.exponential(1.0 / rate, size=total)
    which = rng.integers(0, len(chains.sizes), size=total)
    arrivals = np.cumsum(gaps)
    outstanding = {}
    slot_busy = {}
    rec = []   # (scheduled arrival, submit, admit, start, done, n, status) of measured requests
    done_all = []   # (done, n) of every request, warm-up included
    t0 = time.monotonic_ns()
    sched0 = t0 + 2_000_000
    i = 0
    deadline = time.monotonic() + timeout_s
    while (i < total or outstanding) and time.monotonic() < deadline:
        now = time.monotonic_ns()
        while i < total and sched0 + int(arrivals[i] * 1e9) <= now:
            k = int(which[i])
            j = chains.used[k] % chains.ring
            if (k, j) in slot_busy:   # that step's output buffer is still in use: wait for it
                tk_prev = slot_busy[(k, j)]
                r = server.wait(tk_prev, 60.0)
                _done(outstanding.pop(tk_prev), r, rec, done_all, slot_busy, warmup_n=n_warm)
            chains.used[k] += 1
            tk = server.submit(chains.ds[k], chains.pos[k][j], chains.params[k], prec=prec,
                               grad_x=chains.out[k][j])
            outstanding[tk] = (i, sched0 + int(arrivals[i] * 1e9), chains.sizes[k], (k, j))
            slot_busy[(k, j)] = tk
            i += 1
        for tk in list(outstanding):
            r = server.poll(tk)
            if r is not None:
                _done(outstanding.pop(tk), r, rec, done_all, slot_busy, warmup_n=n_warm)
        time.sleep(100e-6)
    if not rec:
        return {"requests": 0, "offered_rate": rate, "precision": prec, "unfinished": len(outstanding)}
    a = np.array([r[:6] for r in rec], dtype=np.float64)
    st = np.array([r[6] for r in rec])
    lat = (a[:, 4] - a[:, 0]) * 1e-6
    # throughput: every completion (warm-up ones included) inside the window
    # from the first measured arrival to the last measured completion
    w0, w1 = a[:, 0].min(), a[:, 4].max()
    wall = (w1 - w0) * 1e-9
    da = np.array(done_all, dtype=np.float64)
    inside = (da[:, 0] >= w0) & (da[:, 0] <= w1)
    n_in = int(inside.sum())
    pairs_in = float((da[inside, 1] * (da[inside, 1] - 1)).sum())
    sub_wall = (a[:, 1].max() - a[:, 1].min()) * 1e-9

    def pct(v):
        return {"p50": float(np.percentile(v, 50)), "p99": float(np.percentile(v, 99)), "mean": float(v.mean())}

    return {"requests": int(len(rec)), "offered_rate": rate, "precision": prec, "warmup_s": warmup_s,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()),
            "queue_wait_ms": pct((a[:, 2] - a[:, 1]) * 1e-6),
            "admit_to_start_ms": pct((a[:, 3] - a[:, 2]) * 1e-6),
            "service_ms": pct((a[:, 4] - a[:, 3]) * 1e-6),
            "client_lag_ms": pct((a[:, 1] - a[:, 0]) * 1e-6),
            "submit_rate_req_s": (len(rec) - 1) / sub_wall if sub_wall > 0 else None,
            "throughput_req_s": n_in / wall if wall > 0 else None,
            "pairs_per_s": pairs_in / wall if wall > 0 else None,
            "measured_seconds": wall,
            "errors": int((st != 0).sum()), "unfinished": len(outstanding)}


def _done(entry, r, rec, done_all, slot_busy, warmup_n):
    idx, arr_ns, n, slot = entry
    slot_busy.pop(slot, None)
    done_all.append((r["t_done_ns"], n))
    if idx >= warmup_n:
        rec.append((arr_ns, r["t_submit_ns"], r["t_admit_ns"], r["t_start_ns"], r["t_done_ns"], n, r["status"]))
