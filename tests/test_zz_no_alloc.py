"""hawkes_grad_noalloc (workspace in the library's static device scratch)
against hawkes_grad with its own workspace: two calls in a row on the same
scratch, the second with a smaller input, each bitwise equal to hawkes_grad
and within the oracle's tolerance."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2010_02994_amd import _lib, api, workloads as W
from tests.gpu_util import check, oracle_ref, say

pytestmark = pytest.mark.gpu


def _noalloc(x, t, params, prec):
    n, d = x.shape
    gx = torch.full_like(x, float("nan"))
    ll = ctypes.c_double()
    gp = (ctypes.c_double * 6)()
    ps = api.params_struct(params)
    st = _lib.lib().hawkes_grad_noalloc(x.data_ptr(), t.data_ptr(), n, d, ctypes.byref(ps), api._prec(prec),
                                        api._stream_ptr(x.device), ctypes.byref(ll), gx.data_ptr(), gp)
    assert st == _lib.OK, _lib.strerror(st)
    torch.cuda.synchronize()
    return ll.value, gx.cpu().numpy(), np.array(gp[:])


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_matches_grad_two_calls(prec):
    big = W.config1(snapshots=0)                        # N = 10,000
    small = W.random_case(81, 2500, 3, ties=2, t_span=60.0)
    assert _lib.lib().hawkes_workspace_bytes(big.n, big.d, api._prec(prec)) <= 64 << 20
    for w in (big, small):
        say(f"case noalloc {w.name} n={w.n} d={w.d} prec={prec}")
        x = torch.tensor(w.x, device="cuda:0")
        t = torch.tensor(w.t, device="cuda:0")
        a = _noalloc(x, t, w.params, prec)
        ll, gx, gp = api.grad(x, t, w.params, prec=prec)
        b = (ll, gx.cpu().numpy(), gp)
        assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
        check(prec, a, oracle_ref(w.x, w.t, w.params), w.params, label=f"noalloc {w.name}")


def test_noalloc_rejects_sizes_beyond_the_scratch():
    x = torch.zeros((50000, 2), dtype=torch.float64, device="cuda:0")
    t = torch.zeros(50000, dtype=torch.float64, device="cuda:0")
    gx = torch.empty_like(x)
    ps = api.params_struct([0.5, 1, 10, 0.3, 0.1, 2.0])
    say("case noalloc size limit")
    st = _lib.lib().hawkes_grad_noalloc(x.data_ptr(), t.data_ptr(), 50000, 2, ctypes.byref(ps), _lib.MIXED,
                                        api._stream_ptr(x.device), None, gx.data_ptr(), None)
    assert st == _lib.ENOMEM
