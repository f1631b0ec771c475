"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host before any launch."""
import ctypes

import pytest

from paper_2010_02994_amd import _lib


def test_exports_every_declared_symbol():
    L = _lib.lib()
    names = _lib.declared_symbols()
    assert "hawkes_grad" in names and "hawkes_loglik" in names
    for name in names:
        assert hasattr(L, name), name


def test_workspace_bytes_rules():
    L = _lib.lib()
    assert L.hawkes_workspace_bytes(1, 2, 1) == 0
    assert L.hawkes_workspace_bytes(100, 0, 1) == 0
    assert L.hawkes_workspace_bytes(100, 9, 1) == 0
    assert L.hawkes_workspace_bytes(100, 2, 7) == 0
    # the culling flag changes no buffer; other flag bits are rejected
    assert L.hawkes_workspace_bytes(1000, 2, 1 | 0x10) == L.hawkes_workspace_bytes(1000, 2, 1)
    assert L.hawkes_workspace_bytes(1000, 2, 0 | 0x10) == L.hawkes_workspace_bytes(1000, 2, 0)
    assert L.hawkes_workspace_bytes(1000, 2, 1 | 0x20) == 0
    a = L.hawkes_workspace_bytes(50000, 2, 1)
    b = L.hawkes_workspace_bytes(50000, 2, 0)
    assert 0 < a < 1 << 30 and 0 < b < 1 << 30


def test_host_argument_errors():
    L = _lib.lib()
    p = _lib.HawkesParams(0.5, 1, 1, 0.3, 1, 0.5)
    ll = ctypes.c_double(0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the checks fail first
    assert L.hawkes_loglik(None, fake, 10, 2, ctypes.byref(p), 1, fake, 1 << 30, None, ctypes.byref(ll)) == _lib.EINVAL
    assert L.hawkes_loglik(fake, fake, 1, 2, ctypes.byref(p), 1, fake, 1 << 30, None, ctypes.byref(ll)) == _lib.EINVAL
    assert L.hawkes_loglik(fake, fake, 10, 2, ctypes.byref(p), 1, fake, 16, None, ctypes.byref(ll)) == _lib.EINVAL
    for bad in ((0.5, 0, 1, 0.3, 1, 0.5), (0.5, 1, 1, 0.3, -1, 0.5), (0, 1, 1, 0, 1, 0.5),
                (float("nan"), 1, 1, 0.3, 1, 0.5), (-0.1, 1, 1, 0.3, 1, 0.5)):
        pb = _lib.HawkesParams(*bad)
        assert L.hawkes_loglik(fake, fake, 10, 2, ctypes.byref(pb), 1, fake, 1 << 30, None,
                               ctypes.byref(ll)) == _lib.EPARAM
    assert L.hawkes_grad(fake, fake, 10, 2, ctypes.byref(p), 1, fake, 1 << 30, None, None, None, None) == _lib.EINVAL


@pytest.mark.parametrize("code", [0, -1, -2, -3, -4, -5, -6, -7, -8, 1, 99])
def test_strerror(code):
    assert isinstance(_lib.strerror(code), str) and len(_lib.strerror(code)) >= 2


def test_noalloc_rejects_sizes_beyond_its_scratch_on_the_host():
    """hawkes_grad_noalloc refuses (n, d, prec) whose workspace exceeds the
    static scratch before any device call (fake pointers are never touched)."""
    L = _lib.lib()
    p = _lib.HawkesParams(0.5, 1, 10, 0.3, 0.1, 2.0)
    fake = ctypes.c_void_p(0x1000)
    assert L.hawkes_workspace_bytes(50000, 2, 1) > 64 << 20
    assert L.hawkes_grad_noalloc(fake, fake, 50000, 2, ctypes.byref(p), 1, None, None, fake, None) == _lib.ENOMEM
    assert L.hawkes_grad_noalloc(fake, fake, 1, 2, ctypes.byref(p), 1, None, None, fake, None) == _lib.EINVAL
    assert L.hawkes_grad_noalloc(fake, fake, 100, 2, ctypes.byref(p), 1, None, None, None, None) == _lib.EINVAL
