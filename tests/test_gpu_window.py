"""Parity of the moving window of the HIP path with the FP64 oracle.

A jump (one patch column) moves fields and currents, drops the first patch
column's particles, renames every other patch and injects a cold lattice
into the new last column.  Bars: FP64 fields within 1e-11 relative L2, patch
counts, ids and removed counts bit-exact, positions within 1e-11 cells; FP32
within 1e-5 after the steps up to a jump in a weakly driven cold plasma.
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


def _gapped(ncols=400, period=7, value=1.0):
    # a plateau with every period-th column empty (exercises the column skip)
    return np.array([0.0 if c % period == 3 else value for c in range(ncols)])


def _thermal_open(n=(64, 32), patch=(8, 8), ppc=4, T_keV=0.1, seed=5):
    # cells of 1/8, dt = 1/16: one jump every patch[0] * 2 steps at v = 1
    wl = W.uniform_2d(n=n, d=(0.125, 0.125), patch=patch, ppc=ppc, T_keV=T_keV, seed=seed)
    wl["grid"] = dict(wl["grid"], periodic=[0, 1], dt=0.0625)
    return wl


def _pair(wl, precision, window, **kw):
    g = gpu_sim(wl, precision, **kw)
    g.set_window(*window)
    o = oracle.Sim(wl["grid"])
    o.set_particles(wl["x"], wl["u"], wl["w"])
    if wl.get("laser"):
        o.add_laser(wl["laser"])
    o.set_window(*window)
    return g, o


def _check_fp64(g, o, tol=1e-11):
    e, b = compare_fields(g, o)
    assert e < tol and b < tol, (e, b)
    assert np.array_equal(g.counts(), o.counts())
    gx, gu, gw, gid = g.particles()
    ox, ou, ow, oid = o.particles()
    assert np.array_equal(gid, oid)
    for a in range(2):
        assert np.abs(gx[a] - ox[a]).max(initial=0.0) < 1e-11
    assert np.abs(gw - ow).max(initial=0.0) < 1e-15
    d = g.diag()
    assert d["removed"] == o.removed
    assert d["window_cells"] == o.window_shift * g.grid["patch"][0]


def test_window_thermal_fp64_three_jumps():
    _announce("window: open-x thermal 64x32, 8x8 patches, fp64, 50 steps (jumps after 16, 32, 48)")
    wl = _thermal_open()
    g, o = _pair(wl, 64, (0, 1.0, (2, 2), _gapped()))
    g.step(50)
    o.step(50)
    assert o.window_shift == 3
    _check_fp64(g, o)


def test_window_lwfa_fp64_matches_oracle():
    _announce("window: lwfa 512x128 fp64, 70 steps, window from step 5")
    wl = W.lwfa_2d_small(nsteps=70)
    g, o = _pair(wl, 64, (5, 1.0, (2, 2), wl["column_density"]))
    g.step(70)
    o.step(70)
    assert o.window_shift >= 1
    _check_fp64(g, o)


def test_window_fp32_weakly_driven_cold_plasma():
    _announce("window: cold plasma 64x32 fp32 with weak fields, 17 steps (jump after 16)")
    wl = W.to_float32_state(_thermal_open(T_keV=0.0))
    g, o = _pair(wl, 32, (0, 1.0, (2, 2), _gapped(value=0.5)))
    rng = np.random.default_rng(2)
    for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        f = 1e-3 * rng.standard_normal((32, 65)).astype(np.float32).astype(np.float64)
        g.set_field(c, f)
        o.set_field(c, f)
    g.step(17)
    o.step(17)
    assert o.window_shift == 1
    e, b = compare_fields(g, o)
    assert e < 1e-5 and b < 1e-5, (e, b)
    assert np.array_equal(g.counts(), o.counts())
    gx, gu, gw, gid = g.particles()
    ox, ou, ow, oid = o.particles()
    assert np.array_equal(gid, oid)
    assert np.abs(gx[0] - ox[0]).max() < 1e-4 and np.abs(gx[1] - ox[1]).max() < 1e-4


def test_window_in_a_batch_with_graph_replay_and_checkpoint():
    """A windowed simulation stepped in a batch beside a plain one, and a
    windowed simulation replayed from captured graphs and resumed from a
    checkpoint taken after a jump, all against the oracle."""
    _announce("window: batch + graph replay + checkpoint, fp64")
    from paper_1511_03878_amd.sim import Batch, Sim
    wl = _thermal_open(seed=9)
    win = (0, 1.0, (2, 2), _gapped())
    g1, o1 = _pair(wl, 64, win)
    plain = gpu_sim(W.uniform_2d(n=(32, 32), patch=(8, 8), ppc=2), 64)
    b = Batch(64)
    b.add(g1, 40)
    b.add(plain, 40)
    while len(b.finished()) < 2:
        b.step(16)
    b.close()
    o1.step(40)
    _check_fp64(g1, o1)
    # graph replay (32-step graphs) and a checkpoint after the first jump
    g2, o2 = _pair(wl, 64, win, graph=1)
    g2.step(20)
    blob = g2.save_state()
    g3 = Sim(wl["grid"], 64, graph=1)
    g3.load_state(blob)
    g3.set_window(*win)
    g3.step(30)
    o2.step(50)
    _check_fp64(g3, o2)
    g2.step(30)
    _check_fp64(g2, o2)


def test_window_rejects_bad_requests():
    _announce("window: argument checks")
    from paper_1511_03878_amd._capi import PicError
    from paper_1511_03878_amd.sim import Batch
    per = W.uniform_2d(n=(32, 32), patch=(8, 8), ppc=1)
    g = gpu_sim(per, 64)
    with pytest.raises(PicError):
        g.set_window(0, 1.0, (1, 1), [1.0])  # periodic x
    wl = _thermal_open(n=(32, 16), ppc=1)
    g = gpu_sim(wl, 64)
    for bad in ((0, 0.0, (1, 1), [1.0]), (0, 1.5, (1, 1), [1.0]), (-1, 1.0, (1, 1), [1.0]),
                (0, 1.0, (0, 1), [1.0]), (0, 1.0, (1, 1), [-1.0]), (0, 1.0, (1, 1), [np.nan])):
        with pytest.raises(PicError):
            g.set_window(*bad)
    b = Batch(64)
    b.add(g, 1)
    with pytest.raises(PicError):
        g.set_window(0, 1.0, (1, 1), [1.0])
    b.close()


def test_window_full_size_lwfa_conserves_particles():
    """The 4096 x 1024 laser box (FP32) with the window moving from step 50:
    live particles = initial - removed + injected after 200 steps, and the
    window has travelled the cells its speed gives."""
    _announce("window: lwfa 4096x1024 fp32, 200 steps, window from step 50")
    import math
    wl = W.lwfa_2d(nsteps=200)
    g = gpu_sim(wl, 32)
    g.set_window(50, 1.0, (wl["ppc"], 1), wl["column_density"])
    g.step(200)
    d = g.diag()
    dt, dx, P0 = wl["grid"]["dt"], wl["grid"]["d"][0], wl["grid"]["patch"][0]
    jumps = math.floor(1.0 * (200 - 50) * dt / (P0 * dx))
    assert d["window_cells"] == jumps * P0 and jumps >= 3
    _, _, _, ids = g.particles()
    n0 = wl["w"].size
    injected = int(np.count_nonzero(ids >= n0))
    assert d["particles"] == n0 - d["removed"] + injected
    assert injected > 0 and d["flags"] == 0
    assert np.unique(ids).size == ids.size


def test_window_with_merging_and_curve_order_fp64():
    """Merging every 10 steps (before each jump) and the Hilbert-ordered work
    queue together with the window, small laser box, against the oracle."""
    _announce("window + merge every 10 + curve order: lwfa 512x128 fp64, 70 steps")
    wl = W.lwfa_2d_small(nsteps=70, ppc=8)
    win = (5, 1.0, (2, 2), wl["column_density"])
    g, o = _pair(wl, 64, win, patch_order=1)
    g.set_merge(10, 6, 4)
    o.set_merge(10, 6, 4)
    g.step(70)
    o.step(70)
    assert o.window_shift >= 1 and o.merged > 0
    _check_fp64(g, o)
    assert g.diag()["merged"] == o.merged
