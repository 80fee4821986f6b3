"""Parity of the particle merging of the HIP path with the FP64 oracle.

A merge pass on the same state takes the same clustering decisions on both
sides (FP64, the same order of operations), so patch counts and the id of
every slot are bit-exact; FP64 momenta and weights agree to rounding, FP32 to
FP32 rounding.  Merging inside the step loop is checked over 10 FP64 steps
(fields within 1e-11 relative L2).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests import fixtures as W
from tests.helpers import compare_fields, gpu_sim

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _dense(seed, n=(16, 16), patch=(8, 8), maxc=60, umax=5.0):
    rng = np.random.default_rng(seed)
    per_cell = rng.integers(0, maxc, size=n[0] * n[1])
    xs, ys = [], []
    for c, k in enumerate(per_cell):
        xs.append(c % n[0] + rng.uniform(0, 1, k))
        ys.append(c // n[0] + rng.uniform(0, 1, k))
    x = [np.concatenate(xs), np.concatenate(ys)]
    N = x[0].size
    u = [umax * rng.standard_normal(N) for _ in range(3)]
    w = rng.uniform(0.2, 2.0, N)
    grid = dict(ndim=2, n=list(n), d=[0.1, 0.1], dt=0.05, patch=list(patch), periodic=[1, 1], q=-1.0, m=1.0)
    return dict(grid=grid, x=x, u=u, w=w, laser=None)


def _both(wl, precision):
    g = gpu_sim(wl, precision)
    o = oracle.Sim(wl["grid"])
    o.set_particles(wl["x"], wl["u"], wl["w"])
    return g, o


@pytest.mark.parametrize("cmax,iters,seed", [(16, 8, 1), (4, 3, 2), (32, 20, 3)])
def test_merge_pass_fp64_matches_oracle(cmax, iters, seed):
    _announce(f"merge pass fp64 16x16 dense, cmax {cmax}, iters {iters}")
    wl = _dense(seed)
    g, o = _both(wl, 64)
    tg = g.merge(cmax, iters)
    to = o.merge(cmax, iters)
    assert tg == to > 0
    assert np.array_equal(g.counts(), o.counts())
    gx, gu, gw, gid = g.particles()
    ox, ou, ow, oid = o.particles()
    assert np.array_equal(gid, oid)
    for a in range(3):
        np.testing.assert_allclose(gu[a], ou[a], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(gw, ow, rtol=1e-14)
    for a in range(2):
        assert np.abs(gx[a] - ox[a]).max() < 1e-12
    assert g.diag()["merged"] == o.merged


def test_merge_pass_fp32_matches_oracle():
    _announce("merge pass fp32 16x16 dense, cmax 16")
    wl = W.to_float32_state(_dense(5))
    g, o = _both(wl, 32)
    assert g.merge(16, 8) == o.merge(16, 8) > 0
    assert np.array_equal(g.counts(), o.counts())
    gx, gu, gw, gid = g.particles()
    ox, ou, ow, oid = o.particles()
    assert np.array_equal(gid, oid)
    for a in range(3):
        np.testing.assert_allclose(gu[a], ou[a], rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(gw, ow, rtol=2e-7)
    for a in range(2):
        assert np.abs(gx[a] - ox[a]).max() < 1e-5


def test_merge_in_the_step_loop_fp64():
    _announce("merge every 4 steps, thermal 32x32 24ppc fp64, 10 steps")
    wl = W.uniform_2d(n=(32, 32), patch=(8, 8), ppc=24, T_keV=5.0)
    g = gpu_sim(wl, 64)
    g.set_merge(4, 16, 6)
    o = oracle.Sim(wl["grid"])
    o.set_particles(wl["x"], wl["u"], wl["w"])
    o.set_merge(4, 16, 6)
    g.step(10)
    o.step(10)
    assert o.merged > 0 and g.diag()["merged"] == o.merged
    e, b = compare_fields(g, o)
    assert e < 1e-11 and b < 1e-11, (e, b)
    assert np.array_equal(g.counts(), o.counts())
    gx, gu, gw, gid = g.particles()
    ox, ou, ow, oid = o.particles()
    assert np.array_equal(gid, oid)
    for a in range(2):
        assert np.abs(gx[a] - ox[a]).max() < 1e-11


def test_merge_rejects_bad_requests():
    _announce("merge: argument checks")
    from paper_1511_03878_amd._capi import PicError
    from paper_1511_03878_amd.sim import Batch
    g = gpu_sim(_dense(6, maxc=4), 64)
    for bad in ((3, 8), (33, 8), (16, 0), (16, 65)):
        with pytest.raises(PicError):
            g.merge(*bad)
        with pytest.raises(PicError):
            g.set_merge(1, *bad)
    with pytest.raises(PicError):
        g.set_merge(-1)
    wl3 = W.blob_3d(n=(16, 16, 16), patch=(8, 8, 8), ppc0=1, blob_radius=3.0)
    g3 = gpu_sim(wl3, 64)
    with pytest.raises(PicError):
        g3.merge(16, 8)
    b = Batch(64)
    b.add(g, 1)
    with pytest.raises(PicError):
        g.merge(16, 8)
    b.close()
