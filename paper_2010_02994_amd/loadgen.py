"""Open-loop load generator for the serving benchmark (64 HMC chains over
datasets of uneven N, Poisson arrivals).  Each request moves its chain's
latent locations by a small uniform step reflected inside their 100 m cells
(on the device) and asks the server for log-likelihood + gradient there.
Latency runs from the scheduled arrival to completion; the client is never
allowed to hide queueing by submitting late without counting it."""
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


def run(server: Server, chains: Chains, rate: float, n_requests: int, prec: str = "mixed", warmup: int = 50,
        seed: int = 4, want_grad: bool = True, timeout_s: float = 120.0) -> dict:
    rng = np.random.default_rng(seed + 11)
    gaps = rng.exponential(1.0 / rate, size=n_requests + warmup)
    which = rng.integers(0, len(chains.sizes), size=n_requests + warmup)
    arrivals = np.cumsum(gaps)
    outstanding = {}
    lat, pairs_done, statuses = [], 0.0, []
    t0 = time.monotonic_ns()
    sched0 = t0 + 2_000_000
    i = 0
    deadline = time.monotonic() + timeout_s
    while (i < len(arrivals) or outstanding) and time.monotonic() < deadline:
        now = time.monotonic_ns()
        while i < len(arrivals) and sched0 + int(arrivals[i] * 1e9) <= now:
            k = int(which[i])
            x = chains.step(k)
            gx = torch.empty_like(x) if want_grad else None
            torch.cuda.current_stream(chains.dev).synchronize()
            tk = server.submit(chains.ds[k], x, chains.params[k], prec=prec, grad_x=gx)
            outstanding[tk] = (i, sched0 + int(arrivals[i] * 1e9), chains.sizes[k])
            i += 1
        for tk in list(outstanding):
            r = server.poll(tk)
            if r is None:
                continue
            idx, arr_ns, n = outstanding.pop(tk)
            if idx >= warmup:
                lat.append((r["t_done_ns"] - arr_ns) * 1e-6)
                statuses.append(r["status"])
                pairs_done += n * (n - 1)
        time.sleep(50e-6)
    t1 = time.monotonic_ns()
    lat = np.array(lat)
    first_measured = sched0 + int(arrivals[warmup] * 1e9) if len(arrivals) > warmup else t0
    wall = (t1 - first_measured) * 1e-9
    return {"requests": int(len(lat)), "offered_rate": rate, "precision": prec,
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_ms": float(lat.mean()) if len(lat) else None,
            "throughput_req_s": len(lat) / wall if wall > 0 else None,
            "pairs_per_s": pairs_done / wall if wall > 0 else None,
            "errors": int(sum(1 for s in statuses if s != 0)),
            "unfinished": len(outstanding)}
