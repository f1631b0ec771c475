"""Serving scheduler on the CPU (simulate mode: no GPU; requests complete after
a virtual device time).  Admission by slots and HBM footprint, FIFO order,
batching by (D, precision), error paths, drain on destroy."""
import math
import time

import pytest

from paper_2010_02994_amd import _lib
from paper_2010_02994_amd.serve import Server

P = [0.5, 1.0, 1.0, 0.3, 1.0, 0.5]


def _max_concurrent(results):
    ev = []
    for r in results:
        ev.append((r["t_admit_ns"], 1))
        ev.append((r["t_done_ns"], -1))
    ev.sort(key=lambda e: (e[0], e[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def test_slot_limit_bounds_concurrency():
    with Server(hbm_budget_bytes=1 << 30, max_slots=3, streams=4, simulate=True) as s:
        ds = s.register(1, 2, n=20000)
        tks = [s.submit(ds, 1, P) for _ in range(12)]
        res = [s.wait(tk, 10) for tk in tks]
        assert all(r["status"] == 0 for r in res)
        assert _max_concurrent(res) <= 3
        assert s.stats()["batches_launched"] >= 4


def test_memory_budget_bounds_concurrency_and_fifo():
    foot = Server.footprint(20000, 2, "mixed")
    with Server(hbm_budget_bytes=2 * foot + 4096, max_slots=64, streams=4, simulate=True) as s:
        ds = s.register(1, 2, n=20000)
        tks = [s.submit(ds, 1, P) for _ in range(9)]
        res = [s.wait(tk, 10) for tk in tks]
        assert _max_concurrent(res) <= 2
        admits = [r["t_admit_ns"] for r in res]
        assert admits == sorted(admits)          # FIFO admission
        st = s.stats()
        assert st["arena_free_bytes"] == st["arena_bytes"]   # every workspace returned


def test_batches_are_homogeneous_in_dimension_and_precision():
    with Server(hbm_budget_bytes=1 << 30, max_slots=64, streams=1, simulate=True) as s:
        d2 = s.register(1, 2, n=3000)
        d3 = s.register(1, 3, n=3000)
        tks = [s.submit(d2, 1, P, "mixed"), s.submit(d3, 1, P, "mixed"), s.submit(d2, 1, P, "fp64"),
               s.submit(d2, 1, P, "mixed")]
        res = [s.wait(tk, 10) for tk in tks]
        assert all(r["status"] == 0 for r in res)
        # three classes -> at least three batches; the two (d2, mixed) requests may share one
        assert s.stats()["batches_launched"] >= 3


def test_errors_on_submit_and_tickets():
    foot = Server.footprint(5000, 2, "mixed")
    with Server(hbm_budget_bytes=max(foot, 1 << 20) + 4096, max_slots=4, simulate=True) as s:
        ds = s.register(1, 2, n=5000)
        big = s.register(1, 2, n=400000)
        with pytest.raises(_lib.HawkesError) as e:
            s.submit(big, 1, P)
        assert e.value.status == _lib.ENOMEM
        for bad in ([0.5, -1, 1, 0.3, 1, 0.5], [float("nan"), 1, 1, 0.3, 1, 0.5], [0, 1, 1, 0, 1, 0.5]):
            with pytest.raises(_lib.HawkesError) as e:
                s.submit(ds, 1, bad)
            assert e.value.status == _lib.EPARAM
        with pytest.raises(_lib.HawkesError) as e:
            s.submit(99, 1, P)
        assert e.value.status == _lib.ESTATE
        tk = s.submit(ds, 1, P)
        r = s.wait(tk, 10)
        assert r["status"] == 0 and r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_start_ns"] <= r["t_done_ns"]
        with pytest.raises(_lib.HawkesError) as e:
            s.poll(tk)                       # already collected
        assert e.value.status == _lib.ESTATE


def test_wait_timeout_then_poll():
    with Server(hbm_budget_bytes=16 << 30, max_slots=1, streams=1, simulate=True) as s:
        ds = s.register(1, 2, n=300000)       # ~90 ms of virtual device time
        a = s.submit(ds, 1, P)
        b = s.submit(ds, 1, P)
        with pytest.raises(_lib.HawkesError) as e:
            s.wait(b, 0.001)
        assert e.value.status == _lib.ETIMEOUT
        assert s.poll(b) is None               # still pending
        assert s.wait(a, 10)["status"] == 0
        assert s.wait(b, 10)["status"] == 0


def test_destroy_drains_queued_work():
    s = Server(hbm_budget_bytes=1 << 30, max_slots=2, streams=2, simulate=True)
    ds = s.register(1, 2, n=60000)            # ~3.6 ms each
    for _ in range(8):
        s.submit(ds, 1, P)
    t0 = time.perf_counter()
    s.close()                                  # returns only after all 8 completed
    assert time.perf_counter() - t0 >= 4 * 3.6e-3 * 0.9


def test_batches_are_homogeneous_in_the_gradient_flag():
    """Requests with and without a location gradient never share a batch (the
    rate-pass variant depends on it), so with one stream and alternating
    submissions every request starts a batch of its own class."""
    with Server(hbm_budget_bytes=1 << 30, max_slots=64, streams=1, simulate=True) as s:
        d2 = s.register(1, 2, n=3000)
        tks = [s.submit(d2, 1, P, "mixed", grad_x=(1 if k % 2 else None)) for k in range(6)]
        res = [s.wait(tk, 10) for tk in tks]
        assert all(r["status"] == 0 for r in res)
        assert s.stats()["batches_launched"] >= 2


def test_create_with_incomplete_allocator_is_rejected():
    """An allocator without both functions is refused on the host (no device
    call is made)."""
    import ctypes
    from paper_2010_02994_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    spec = _lib.HawkesAllocator()   # both function pointers NULL
    st = L.hawkes_serve_create_with(ctypes.byref(spec), 1 << 30, 4, _lib.SERVE_SIMULATE, ctypes.byref(h))
    assert st == _lib.EINVAL and not h.value


def test_batches_group_by_size_band():
    """Requests of one class but N a factor of 20 apart go to different
    batches (a batch ends with its largest request), each batch starting all
    of its requests together."""
    with Server(hbm_budget_bytes=8 << 30, max_slots=64, streams=1, simulate=True) as s:
        big = s.register(1, 2, n=200000)
        small = s.register(1, 2, n=2000)
        large = s.register(1, 2, n=40000)
        blocker = s.submit(big, 1, P)           # holds the only stream for ~40 ms
        tks = [s.submit(small if k % 2 == 0 else large, 1, P) for k in range(8)]
        assert s.wait(blocker, 10)["status"] == 0
        res = [s.wait(tk, 10) for tk in tks]
        assert all(r["status"] == 0 for r in res)
        starts_small = {r["t_start_ns"] for r in res[0::2]}
        starts_large = {r["t_start_ns"] for r in res[1::2]}
        assert len(starts_small) == 1 and len(starts_large) == 1 and starts_small != starts_large
        assert s.stats()["batches_launched"] == 3
