"""Longer GPU checks: FP32 charge continuity and energy drift, and the full
4096 x 1024 laser-wakefield box in the launch configuration bench.py times."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

from tests import fixtures as W
from tests.brute import div_dual_2d
from tests.helpers import compare_fields, gpu_sim, oracle_run

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _rho_numpy(x, y, w, q, n):
    """Charge density on primal nodes of a periodic grid (quadratic shapes),
    accumulated in FP64 with numpy (independent of both implementations)."""
    rho = np.zeros((n[1], n[0]))
    ix = np.floor(x + 0.5).astype(np.int64)
    iy = np.floor(y + 0.5).astype(np.int64)
    dx, dy = x - ix, y - iy
    wx = [0.5 * (0.5 - dx) ** 2, 0.75 - dx ** 2, 0.5 * (0.5 + dx) ** 2]
    wy = [0.5 * (0.5 - dy) ** 2, 0.75 - dy ** 2, 0.5 * (0.5 + dy) ** 2]
    for b in range(3):
        for a in range(3):
            np.add.at(rho, ((iy + b - 1) % n[1], (ix + a - 1) % n[0]), q * w * wx[a] * wy[b])
    return rho


def test_fp32_charge_continuity_residual():
    _announce("fp32 continuity residual, 64x64 16ppc 10 keV")
    wl = W.to_float32_state(W.uniform_2d(n=(64, 64), patch=(16, 16), ppc=16, T_keV=10.0))
    g = gpu_sim(wl, 32)
    g.step(5)
    x0, _, w0, id0 = g.particles()
    g.step(1)
    x1, _, w1, id1 = g.particles()
    n = wl["grid"]["n"]
    d = wl["grid"]["d"]
    dt = wl["grid"]["dt"]
    r0 = _rho_numpy(x0[0], x0[1], w0, -1.0, n)
    r1 = _rho_numpy(x1[0], x1[1], w1, -1.0, n)
    Jx, Jy = g.field("Jx"), g.field("Jy")
    res = np.abs(r1 - r0 + dt * div_dual_2d(Jx, Jy, d)).max() / np.abs(r0).max()
    assert res < 1e-6, res


def test_fp32_energy_drift_follows_oracle_over_1000_steps():
    _announce("fp32 uniform 128x128, 1000 steps, energy drift vs oracle history")
    with open(os.path.join(GOLDEN, "energy_uniform_1000.json")) as f:
        gold = json.load(f)
    wl = W.to_float32_state(W.uniform_2d())
    g = gpu_sim(wl, 32)
    g.step(1000)
    U, K, _ = g.history(0, 1000)
    Wg = U + K
    Wo = np.array(gold["U"]) + np.array(gold["K"])
    # the drift itself is the scheme's numerical heating of this box (the
    # FP64 oracle drifts by 1.5e-3 too); the FP32 history must follow the
    # oracle's closely at every step, not only in its end value
    drift_g = (Wg[-1] - Wg[0]) / Wg[0]
    drift_o = (Wo[-1] - Wo[0]) / Wo[0]
    err = np.abs(Wg - Wo).max() / Wo[0]
    print(f"[gpu-test] drift fp32 {drift_g:.6e} oracle {drift_o:.6e}, max |W - W_oracle| / W0 {err:.3e}",
          flush=True)
    # measured: drift 1.4773e-3 against the oracle's 1.4769e-3, history within 6.4e-7 of W0
    assert abs(drift_g - drift_o) < 1e-5, (drift_g, drift_o)
    assert err < 1e-5, err


def test_full_lwfa_box_one_step_fp32_and_invariants():
    """The 4096 x 1024 box (16.5 M particles) in bench.py's configuration: one
    step against the oracle, then particle conservation over 100 steps."""
    _announce("lwfa 4096x1024 fp32: 1 step vs oracle, 100 steps invariants")
    wl = W.to_float32_state(W.lwfa_2d(nsteps=120))
    g = gpu_sim(wl, 32)
    g.step(1)
    o = oracle_run(wl, 1)
    e, b = compare_fields(g, o)
    assert e < 1e-5 and b < 1e-5, (e, b)
    assert np.array_equal(g.counts(), o.counts())
    del o
    g.step(99)
    d = g.diag()
    assert d["step"] == 100
    assert d["particles"] + d["removed"] == wl["w"].size
    assert d["flags"] == 0
    # the laser has entered: field energy grows while the pulse is driven in
    U, K, P = g.history(0, 100)
    assert U[-1] > U[10] > 0.0
    assert np.all(P[:100] + 0 <= wl["w"].size)
