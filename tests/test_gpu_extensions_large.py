"""The sixth-order solver and merging at large sizes against the FP64 oracle:
the sixth-order field update on the full 4096 x 1024 grid, the FP32 energy
history of the thermal box over 1000 sixth-order steps against the oracle's
stored history, and a merge pass over 4096 patches (more patches than the
merge kernel has workgroups)."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import oracle
from tests import fixtures as W
from tests.helpers import compare_fields, gpu_sim

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
S6 = 75 / 64 + 25 / 384 + 3 / 640


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def test_sixth_order_full_grid_fields():
    _announce("sixth-order vacuum fields 4096x1024: fp64 2 steps, fp32 1 step")
    from paper_1511_03878_amd.sim import Sim
    n, d = (4096, 1024), (0.1, 0.1)
    grid = dict(ndim=2, n=list(n), d=list(d), dt=W.cfl_dt(d, 0.9 / S6), patch=[32, 32],
                periodic=[1, 1], q=-1.0, m=1.0)
    rng = np.random.default_rng(41)
    F = [rng.standard_normal((n[1], n[0])).astype(np.float32).astype(np.float64) for _ in range(6)]
    o = oracle.Sim(grid)
    o.set_maxwell_order(6)
    for c, f in zip(("Ex", "Ey", "Ez", "Bx", "By", "Bz"), F):
        o.set_field(c, f)
    o.step(1)
    for prec, steps, tol in ((32, 1, 1e-5), (64, 2, 1e-12)):
        g = Sim(grid, prec, maxwell_order=6)
        g.set_particles([np.zeros(0), np.zeros(0)], [np.zeros(0)] * 3, np.zeros(0))
        for c, f in zip(("Ex", "Ey", "Ez", "Bx", "By", "Bz"), F):
            g.set_field(c, f)
        g.step(steps)
        if steps == 2:
            o.step(1)
        e, b = compare_fields(g, o)
        assert e < tol and b < tol, (prec, e, b)
        g.close()


def test_sixth_order_fp32_energy_drift_follows_oracle_over_1000_steps():
    _announce("fp32 uniform 128x128 sixth order, 1000 steps, energy drift vs oracle history")
    with open(os.path.join(GOLDEN, "energy_uniform_1000_order6.json")) as f:
        gold = json.load(f)
    wl = W.to_float32_state(W.uniform_2d(cfl=0.95 / S6))
    g = gpu_sim(wl, 32, maxwell_order=6)
    g.step(1000)
    U, K, _ = g.history(0, 1000)
    Wg = U + K
    Wo = np.array(gold["U"]) + np.array(gold["K"])
    drift_g = (Wg[-1] - Wg[0]) / Wg[0]
    drift_o = (Wo[-1] - Wo[0]) / Wo[0]
    assert abs(drift_g - drift_o) < 1e-3, (drift_g, drift_o)
    assert np.abs(Wg - Wo).max() / Wo[0] < 1e-3


def test_merge_pass_over_4096_patches_fp64():
    _announce("merge pass fp64, 512x512 cells, 8x8 patches (4096), 20 ppc, cmax 16")
    wl = W.uniform_2d(n=(512, 512), patch=(8, 8), ppc=20, T_keV=10.0, seed=77)
    g = gpu_sim(wl, 64)
    o = oracle.Sim(wl["grid"])
    o.set_particles(wl["x"], wl["u"], wl["w"])
    assert g.merge(16, 6) == o.merge(16, 6) > 0
    assert np.array_equal(g.counts(), o.counts())
    gx, gu, gw, gid = g.particles()
    ox, ou, ow, oid = o.particles()
    assert np.array_equal(gid, oid)
    for a in range(3):
        np.testing.assert_allclose(gu[a], ou[a], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(gw, ow, rtol=1e-14)


def test_merge_pass_with_more_members_than_the_lds_copy_fp64():
    """Patches of 64 x 64 cells at 9 per cell: more crowded-cell members per
    patch (36864) than the kernel keeps in LDS, so the clusters are read back
    from the particle codes; same result as the oracle."""
    _announce("merge pass fp64, 128x128 cells, 64x64 patches, 9 ppc, cmax 4")
    wl = W.uniform_2d(n=(128, 128), patch=(64, 64), ppc=9, T_keV=10.0, seed=78)
    g = gpu_sim(wl, 64)
    o = oracle.Sim(wl["grid"])
    o.set_particles(wl["x"], wl["u"], wl["w"])
    assert g.merge(4, 3) == o.merge(4, 3) > 0
    assert np.array_equal(g.counts(), o.counts())
    gx, gu, gw, gid = g.particles()
    ox, ou, ow, oid = o.particles()
    assert np.array_equal(gid, oid)
    for a in range(3):
        np.testing.assert_allclose(gu[a], ou[a], rtol=1e-13, atol=1e-13)
