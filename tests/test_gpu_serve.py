"""Serving on the GPU: every result identical alone and in the mix (bitwise),
identical to the direct C ABI call, within tolerance of the oracle; a bad
request fails alone; a short open-loop run completes without errors."""
import numpy as np
import pytest
import torch

import oracle
from paper_2010_02994_amd import _lib, api, workloads as W
from paper_2010_02994_amd.serve import Server
from tests.gpu_util import check, oracle_ref, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SIZES = [700, 1500, 3000, 5000, 2000, 12000]


@pytest.fixture(scope="module")
def data():
    out = []
    for k, n in enumerate(SIZES):
        w = W.serving_dataset(k, n)
        out.append((w, torch.tensor(w.x, device=DEV), torch.tensor(w.t, device=DEV)))
    return out


def _run_set(server, ids, data, reqs, together):
    """reqs: list of (dataset index, prec).  Returns [(status, ll, gp, grad_x numpy)].
    Together: a float64 request on the largest dataset is submitted first and
    holds the server's stream while the others queue, so they are batched
    whatever the host's submission speed."""
    outs = [torch.full_like(data[k][1], float("nan")) for k, _ in reqs]
    res = [None] * len(reqs)
    if together:
        big = max(range(len(data)), key=lambda k: data[k][0].n)
        blocker = server.submit(ids[big], data[big][1], data[big][0].params, prec="fp64",
                                grad_x=torch.empty_like(data[big][1]))
        tks = [server.submit(ids[k], data[k][1], data[k][0].params, prec=p, grad_x=outs[j])
               for j, (k, p) in enumerate(reqs)]
        assert server.wait(blocker, 60)["status"] == 0
        for j, tk in enumerate(tks):
            res[j] = server.wait(tk, 60)
    else:
        for j, (k, p) in enumerate(reqs):
            res[j] = server.wait(server.submit(ids[k], data[k][1], data[k][0].params, prec=p, grad_x=outs[j]), 60)
    torch.cuda.synchronize()
    return [(r["status"], r["loglik"], np.array(r["grad_params"]), o.cpu().numpy()) for r, o in zip(res, outs)]


def test_alone_vs_mix_bitwise_and_direct_call(data):
    reqs = [(k, p) for k in range(len(SIZES)) for p in ("mixed", "fp64")]
    with Server(hbm_budget_bytes=4 << 30, max_slots=64, streams=1) as s:
        ids = [s.register(d[2], 2) for d in data]
        say("case serve alone")
        alone = _run_set(s, ids, data, reqs, together=False)
        say("case serve mix")
        mix = _run_set(s, ids, data, reqs, together=True)
        st = s.stats()
    # alone: one batch per request; the mix (after the blocker) shares batches
    assert st["batches_launched"] < len(reqs) * 2 + 1
    for (k, p), a, m in zip(reqs, alone, mix):
        assert a[0] == 0 and m[0] == 0
        assert a[1] == m[1] and np.array_equal(a[2], m[2]) and np.array_equal(a[3], m[3]), (k, p)
        w, x, t = data[k]
        ll, gx, gp = api.grad(x, t, w.params, prec=p)
        assert ll == a[1] and np.array_equal(gp, a[2]) and np.array_equal(gx.cpu().numpy(), a[3]), (k, p)
    for k in (0, 3):
        w = data[k][0]
        ref = oracle_ref(w.x, w.t, w.params)
        for p in ("mixed", "fp64"):
            j = reqs.index((k, p))
            check(p, (alone[j][1], alone[j][3], alone[j][2]), ref, w.params, label=f"serve{k}")


def test_requests_without_gradient_match_the_direct_call(data):
    """Requests with no location gradient (log-likelihood and parameter
    gradients only), submitted interleaved with gradient requests, equal the
    direct enqueue-only call with grad_x = NULL bit for bit."""
    with Server(hbm_budget_bytes=4 << 30, max_slots=64, streams=3) as s:
        ids = [s.register(d[2], 2) for d in data]
        say("case serve requests without gradient")
        outs = {k: torch.full_like(data[k][1], float("nan")) for k in (0, 3)}
        plan = [(0, None), (1, None), (0, "g"), (3, None), (3, "g"), (2, None)]
        tks = [s.submit(ids[k], data[k][1], data[k][0].params, prec="mixed",
                        grad_x=(outs[k] if g else None)) for k, g in plan]
        res = [s.wait(tk, 60) for tk in tks]
    torch.cuda.synchronize()
    for (k, g), r in zip(plan, res):
        w, x, t = data[k]
        assert r["status"] == 0
        if g:
            ll, gx, gp = api.grad(x, t, w.params, prec="mixed")
            assert np.array_equal(gx.cpu().numpy(), outs[k].cpu().numpy()), k
        else:
            out8 = api.grad_async(x, t, w.params, prec="mixed").cpu().numpy()
            ll, gp = out8[0], out8[1:7]
        assert r["loglik"] == ll and np.array_equal(np.array(r["grad_params"]), gp), (k, g)


def test_bad_request_fails_alone(data):
    with Server(hbm_budget_bytes=2 << 30, max_slots=16) as s:
        ids = [s.register(d[2], 2) for d in data]
        bad_x = data[2][1].clone()
        bad_x[10, 0] = float("nan")
        say("case serve failure isolation")
        good = [s.submit(ids[k], data[k][1], data[k][0].params, prec="mixed") for k in (0, 1, 3)]
        bad = s.submit(ids[2], bad_x, data[2][0].params, prec="mixed")
        more = [s.submit(ids[k], data[k][1], data[k][0].params, prec="mixed") for k in (4, 5)]
        rb = s.wait(bad, 60)
        assert rb["status"] == _lib.EDATA
        for tk, k in zip(good + more, (0, 1, 3, 4, 5)):
            r = s.wait(tk, 60)
            assert r["status"] == 0
            ll = api.loglik(data[k][1], data[k][2], data[k][0].params, prec="mixed")
            assert r["loglik"] == ll


def test_tight_budget_still_completes(data):
    foot = Server.footprint(12000, 2, "mixed")
    with Server(hbm_budget_bytes=foot + (1 << 20), max_slots=8) as s:
        ids = [s.register(d[2], 2) for d in data]
        say("case serve tight budget")
        tks = [s.submit(ids[k], data[k][1], data[k][0].params, prec="mixed") for k in range(len(SIZES))] * 1
        res = [s.wait(tk, 60) for tk in tks]
        assert all(r["status"] == 0 for r in res)
        st = s.stats()
        assert st["arena_free_bytes"] == st["arena_bytes"]


def test_open_loop_short_run():
    from paper_2010_02994_amd import loadgen
    with Server(hbm_budget_bytes=16 << 30, max_slots=64, streams=2) as s:
        say("case serve open loop")
        chains = loadgen.Chains(s, count=16, lo=1e3, hi=2e4)
        out = loadgen.run(s, chains, rate=200.0, n_requests=200, prec="mixed", warmup_s=0.1)
    say(f"  open loop: {out}")
    assert out["requests"] == 200 and out["errors"] == 0 and out["unfinished"] == 0
    assert out["p50_ms"] > 0 and out["p99_ms"] >= out["p50_ms"]


def test_server_on_torch_memory(data):
    """A server whose arena, result slots and dataset copies come from
    PyTorch's caching allocator gives the direct call's results bitwise, holds
    its blocks while open (torch accounts for the arena) and gives every block
    back when closed."""
    budget = 1 << 30
    before = torch.cuda.memory_allocated()
    with Server(hbm_budget_bytes=budget, max_slots=16, streams=2, torch_memory=True) as s:
        ids = [s.register(d[2], 2) for d in data[:3]]
        say("case serve on torch memory")
        assert s.device_blocks() == 1 + 2 * 2 + 3
        assert torch.cuda.memory_allocated() - before >= budget
        outs = [torch.full_like(data[k][1], float("nan")) for k in range(3)]
        res = [s.wait(s.submit(ids[k], data[k][1], data[k][0].params, prec="mixed", grad_x=outs[k]), 60)
               for k in range(3)]
        torch.cuda.synchronize()
        for k, r in enumerate(res):
            w, x, t = data[k]
            ll, gx, gp = api.grad(x, t, w.params, prec="mixed")
            assert r["status"] == 0 and r["loglik"] == ll and np.array_equal(np.array(r["grad_params"]), gp)
            assert np.array_equal(outs[k].cpu().numpy(), gx.cpu().numpy())
    assert s.device_blocks() == 0
