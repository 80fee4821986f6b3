"""The optional passes under graph replay and in mixed batches, against the
FP64 oracle: merging and the sixth-order solver replayed from captured
32-step graphs, and a 3-D batch holding a Yee and a sixth-order box."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests import fixtures as W
from tests.helpers import compare_fields, gpu_sim

pytestmark = pytest.mark.gpu

S6 = 75 / 64 + 25 / 384 + 3 / 640


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _check(g, o, tol=1e-11):
    e, b = compare_fields(g, o)
    assert e < tol and b < tol, (e, b)
    assert np.array_equal(g.counts(), o.counts())
    assert np.array_equal(g.particles()[3], o.particles()[3])


def test_merging_replayed_from_graphs_fp64():
    _announce("merge every 4 steps under graph replay, thermal 32x32 24ppc fp64, 40 steps")
    wl = W.uniform_2d(n=(32, 32), patch=(8, 8), ppc=24, T_keV=5.0, seed=12)
    g = gpu_sim(wl, 64, graph=1)
    g.set_merge(4, 16, 6)
    o = oracle.Sim(wl["grid"])
    o.set_particles(wl["x"], wl["u"], wl["w"])
    o.set_merge(4, 16, 6)
    g.step(40)
    o.step(40)
    assert o.merged > 0 and g.diag()["merged"] == o.merged
    _check(g, o)


def test_sixth_order_replayed_from_graphs_fp64():
    _announce("sixth-order thermal 64x64 under graph replay fp64, 40 steps")
    wl = W.uniform_2d(n=(64, 64), ppc=4, T_keV=0.2, cfl=0.95 / S6, seed=13)
    g = gpu_sim(wl, 64, graph=1, maxwell_order=6)
    o = oracle.Sim(wl["grid"])
    o.set_maxwell_order(6)
    o.set_particles(wl["x"], wl["u"], wl["w"])
    g.step(40)
    o.step(40)
    _check(g, o, 1e-10)


def test_3d_batch_with_yee_and_sixth_order_fp64():
    _announce("3-D batch: Yee box and sixth-order box, vacuum fields fp64, 8 steps")
    from paper_1511_03878_amd.sim import Batch, Sim
    sims = []
    for order, n, seed in ((2, (16, 16, 16), 1), (6, (24, 16, 16), 2)):
        d = (0.1, 0.1, 0.1)
        grid = dict(ndim=3, n=list(n), d=list(d), dt=W.cfl_dt(d, 0.9 / S6), patch=[8, 8, 8],
                    periodic=[1, 1, 1], q=-1.0, m=1.0)
        g = Sim(grid, 64, maxwell_order=order)
        g.set_particles([np.zeros(0)] * 3, [np.zeros(0)] * 3, np.zeros(0))
        o = oracle.Sim(grid)
        if order == 6:
            o.set_maxwell_order(6)
        rng = np.random.default_rng(seed)
        for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
            f = rng.standard_normal((n[2], n[1], n[0]))
            g.set_field(c, f)
            o.set_field(c, f)
        sims.append((g, o))
    b = Batch(64, ndim=3)
    for g, _ in sims:
        b.add(g, 8)
    while len(b.finished()) < 2:
        b.step(16)
    b.close()
    for g, o in sims:
        o.step(8)
        e, bb = compare_fields(g, o)
        assert e < 1e-12 and bb < 1e-12, (e, bb)


def test_autotune_with_window_and_merging_restores_state(tmp_path):
    """The tuner's trial steps jump the window and merge; the state it
    restores afterwards is the one it started from, and the run then
    continues to agree with the oracle (FP64)."""
    _announce("autotune with window + merging, lwfa 512x128 fp64")
    wl = W.lwfa_2d_small(nsteps=200, ppc=8)
    win = (0, 1.0, (2, 2), wl["column_density"])
    g = gpu_sim(wl, 64)
    g.set_window(*win)
    g.set_merge(5, 6, 4)
    o = oracle.Sim(wl["grid"])
    o.set_particles(wl["x"], wl["u"], wl["w"])
    o.add_laser(wl["laser"])
    o.set_window(*win)
    o.set_merge(5, 6, 4)
    g.step(30)
    before = g.save_state()
    g.autotune(steps=40, cache=str(tmp_path / "tune.txt"))
    assert g.save_state() == before
    g.step(20)
    o.step(50)
    assert o.window_shift >= 1 and o.merged > 0
    _check(g, o)
    assert g.diag()["removed"] == o.removed
