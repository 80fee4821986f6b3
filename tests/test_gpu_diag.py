"""Diagnostics on the GPU: the charge density (2-D and 3-D) against numpy's
quadratic-shape accumulation, and the library's Gauss and continuity residuals
against the same residuals evaluated in numpy from the GPU's own positions,
fields and currents."""
from __future__ import annotations

import math

import numpy as np
import pytest

from tests import fixtures as W
from tests.brute import div_dual_2d, rho_2d, rho_3d
from tests.helpers import gpu_sim

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _div_e_2d(g, d):
    return div_dual_2d(g.field("Ex"), g.field("Ey"), d)


def _div3(F, d):
    return sum((F[a] - np.roll(F[a], 1, axis=2 - a)) / d[a] for a in range(3))


@pytest.mark.parametrize("precision", [64, 32])
def test_rho_2d_matches_numpy(precision):
    _announce(f"rho 2-D fp{precision}")
    wl = W.uniform_2d(n=(64, 32), patch=(16, 16), ppc=8, T_keV=10.0)
    g = gpu_sim(wl, precision)
    g.step(3)
    x, _, w, _ = g.particles()
    n = wl["grid"]["n"]
    ref = rho_2d(x[0], x[1], w, -1.0, n)
    got = g.field("rho")
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_rho_3d_matches_numpy():
    _announce("rho 3-D fp64")
    wl = W.blob_3d(n=(32, 16, 16), patch=(8, 8, 4), T_keV=20.0, ppc0=2)
    g = gpu_sim(wl, 64)
    g.step(2)
    x, _, w, _ = g.particles()
    ref = rho_3d(x, w, -1.0, wl["grid"]["n"])
    got = g.field("rho")
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("precision,tol", [(64, 1e-12), (32, 1e-6)])
def test_residuals_2d_periodic(precision, tol):
    _announce(f"residuals 2-D periodic fp{precision}")
    wl = W.uniform_2d(n=(64, 64), patch=(16, 16), ppc=16, T_keV=10.0)
    if precision == 32:
        wl = W.to_float32_state(wl)
    g = gpu_sim(wl, precision)
    r0 = g.residuals()
    assert r0["step"] == 0 and math.isnan(r0["continuity"])
    # E = 0 and rho = rho^0 at load, up to the order of the FP64 atomic sums
    # of rho (16 particles x 9 nodes of same-sign terms per node: relative
    # difference below 144 x 2^-53 = 1.6e-14)
    assert r0["gauss"] <= 2e-14
    g.step(5)
    x0, _, w0, _ = g.particles()
    ra = g.residuals()
    g.step(1)
    x1, _, w1, _ = g.particles()
    rb = g.residuals()
    assert rb["step"] == 6 and not math.isnan(rb["continuity"])
    n, d, dt = wl["grid"]["n"], wl["grid"]["d"], wl["grid"]["dt"]
    if precision == 32:
        # the FP32 kernels (and the library's residuals) use the cell size and
        # time step as stored in FP32
        d, dt = [float(np.float32(v)) for v in d], float(np.float32(dt))
    rho0 = rho_2d(wl["x"][0], wl["x"][1], wl["w"], -1.0, n)
    rho_a = rho_2d(x0[0], x0[1], w0, -1.0, n)
    rho_b = rho_2d(x1[0], x1[1], w1, -1.0, n)
    cont = np.abs(rho_b - rho_a + dt * div_dual_2d(g.field("Jx"), g.field("Jy"), d)).max()
    cont /= np.abs(rho_b).max()
    gauss = np.abs(_div_e_2d(g, d) - (rho_b - rho0)).max() / np.abs(rho0).max()
    assert rb["continuity"] < tol and rb["gauss"] < 100 * tol
    assert abs(rb["continuity"] - cont) <= 1e-9
    assert abs(rb["gauss"] - gauss) <= 1e-9 + 1e-6 * gauss
    assert abs(rb["rho_max"] - np.abs(rho_b).max()) <= 1e-12 * rb["rho_max"]
    assert ra["step"] == 5 and math.isnan(ra["continuity"])  # no call at step 4


def test_residuals_3d_fp64():
    _announce("residuals 3-D fp64")
    wl = W.blob_3d(n=(32, 16, 16), patch=(8, 8, 4), T_keV=50.0, ppc0=2)
    g = gpu_sim(wl, 64)
    g.step(3)
    x0, _, w0, _ = g.particles()
    g.residuals()
    g.step(1)
    x1, _, w1, _ = g.particles()
    r = g.residuals()
    n, d, dt = wl["grid"]["n"], wl["grid"]["d"], wl["grid"]["dt"]
    rho_a, rho_b = rho_3d(x0, w0, -1.0, n), rho_3d(x1, w1, -1.0, n)
    J = [g.field(c) for c in ("Jx", "Jy", "Jz")]
    E = [g.field(c) for c in ("Ex", "Ey", "Ez")]
    rho0 = rho_3d(wl["x"], wl["w"], -1.0, n)
    cont = np.abs(rho_b - rho_a + dt * _div3(J, d)).max() / np.abs(rho_b).max()
    gauss = np.abs(_div3(E, d) - (rho_b - rho0)).max() / np.abs(rho0).max()
    assert r["continuity"] < 1e-12 and r["gauss"] < 1e-11
    assert abs(r["continuity"] - cont) <= 1e-13
    assert abs(r["gauss"] - gauss) <= 1e-13


def test_residuals_open_box_and_checkpoint():
    """Laser box (open x): the residuals leave out the nodes next to the faces;
    after a checkpoint load the Gauss reference is unknown (NaN)."""
    _announce("residuals small laser box fp64 + checkpoint")
    wl = W.lwfa_2d_small(nsteps=80)
    g = gpu_sim(wl, 64)
    g.step(70)
    g.residuals()
    g.step(1)
    r = g.residuals()
    assert r["continuity"] < 1e-12 and r["gauss"] < 1e-10, r
    blob = g.save_state()
    h = gpu_sim(wl, 64)
    h.load_state(blob)
    r2 = h.residuals()
    assert math.isnan(r2["gauss"]) and math.isnan(r2["continuity"])
    assert r2["rho_max"] == pytest.approx(r["rho_max"], rel=1e-14)


def test_imbalance_from_item_stamps():
    """pic_imbalance on the small laser box once the pulse is in the plasma:
    every item is stamped, the work queue spreads the item time more evenly
    over the compute units than fixed domains of equal patch-id runs would,
    and the accounting adds up."""
    _announce("imbalance from item stamps, small laser box fp32")
    from paper_1511_03878_amd._capi import PicError
    wl = W.lwfa_2d_small()
    g = gpu_sim(wl, 32)
    g.step(60)
    with pytest.raises(PicError) as e:
        g.imbalance()
    assert e.value.code == -8
    g.timing_enable("stamps")
    g.step(1)
    r = g.imbalance()
    g.timing_enable(False)
    assert r["step"] == 61 and r["items"] >= 1 and 1 <= r["units"] <= r["device_units"]
    assert r["imbalance"] >= 1.0 and r["static_imbalance"] >= r["imbalance"]
    assert r["segment_imbalance"] >= 1.0
    total = r["busy_mean_us"] * r["device_units"]
    assert total == pytest.approx(r["patch_mean_us"] * g.npatch, rel=1e-9)
    assert r["span_us"] > 0 and r["busy_max_us"] <= r["span_us"] * 64
