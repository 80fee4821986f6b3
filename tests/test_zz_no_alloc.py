"""The allocation-free charge density (pic_rho_get_noalloc) against the
allocating pic_fields_get(PIC_RHO), called through the C-ABI: two calls in a
row on one GPU, the second on a smaller grid, and the size checks."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from paper_1511_03878_amd import _capi
from tests import fixtures as W
from paper_1511_03878_amd.sim import Sim
from tests.helpers import gpu_sim

pytestmark = pytest.mark.gpu
_DP = C.POINTER(C.c_double)


def _noalloc(sim, n, buf=None):
    out = np.full(n, np.nan) if buf is None else buf
    rc = _capi.load().pic_rho_get_noalloc(sim.handle, out.ctypes.data_as(_DP), n)
    return rc, out


def _rho_alloc(sim, n):
    out = np.zeros(n)
    _capi.check(_capi.load().pic_fields_get(sim.handle, 9, out.ctypes.data_as(_DP), n))
    return out


def test_noalloc_rho_matches_the_allocating_call():
    print("[gpu-test] pic_rho_get_noalloc vs pic_fields_get(rho): 2-D fp64 then smaller 3-D fp32",
          flush=True)
    cases = [(W.uniform_2d(n=(256, 128), patch=(16, 16), ppc=8, T_keV=10.0), 64, 4),
             (W.blob_3d(n=(16, 16, 8), patch=(8, 8, 4), T_keV=20.0, ppc0=2), 32, 2)]
    sizes = []
    for wl, prec, steps in cases:
        g = gpu_sim(wl, prec)
        g.step(steps)
        n = int(np.prod(g.fn))
        sizes.append(n)
        ref = _rho_alloc(g, n)
        scale = np.abs(ref).max()
        assert scale > 0
        rc, got = _noalloc(g, n)
        assert rc == 0, _capi.load().pic_last_error()
        assert np.abs(got - ref).max() <= 1e-13 * scale
        # the same state again: the scratch is cleared on every call
        rc, again = _noalloc(g, n)
        assert rc == 0 and np.abs(again - ref).max() <= 1e-13 * scale
        g.close()
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_a_bad_count_and_an_oversized_grid():
    print("[gpu-test] pic_rho_get_noalloc argument checks", flush=True)
    wl = W.uniform_2d(n=(64, 32), patch=(16, 16), ppc=2)
    g = gpu_sim(wl, 64)
    n = int(np.prod(g.fn))
    rc, _ = _noalloc(g, n - 1, np.zeros(n))
    assert rc == -1  # PIC_EINVAL
    g.close()
    grid = dict(ndim=2, n=[4096, 2112], d=[0.1, 0.1], dt=0.05, patch=[32, 32], periodic=[1, 1],
                q=-1.0, m=1.0)
    big = Sim(grid, 32)
    nbig = 4096 * 2112  # periodic axes: one node per cell
    assert nbig > 8388608
    rc, _ = _noalloc(big, nbig, np.zeros(nbig))
    assert rc == -1
    assert "allocation-free scratch" in _capi.load().pic_last_error().decode()
    big.close()
