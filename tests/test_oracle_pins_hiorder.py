"""Pins of the oracle's sixth-order field solver (no GPU).

The coefficients are derived here from their defining Taylor conditions (not
copied from the oracle); the oracle's update must then carry discrete plane
waves exactly at the frequency of the dispersion relation of that stencil,
sin(w dt / 2) = (dt / 2) |k~|, k~_a = (2 / d_a) sum_m c_m sin((2m - 1) k_a d_a / 2),
in 2-D and 3-D, and keep the sixth-order divergence of B at rounding level.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from tests import fixtures as W
from tests import brute


def _coefficients():
    # sum_m c_m (2m - 1)^p = 1 for p = 1 and 0 for p = 3, 5
    A = np.array([[(2 * m - 1) ** p for m in (1, 2, 3)] for p in (1, 3, 5)], dtype=float)
    return np.linalg.solve(A, np.array([1.0, 0.0, 0.0]))


C6 = _coefficients()


def _mod_sin(k, d):
    """S = sum_m c_m sin((2m - 1) k d / 2), so that k~ = 2 S / d."""
    return sum(C6[m - 1] * math.sin((2 * m - 1) * k * d / 2) for m in (1, 2, 3))


def _dfw(f, axis, d):
    """Sixth-order forward staggered difference along a numpy axis (periodic)."""
    return sum(C6[m - 1] * (np.roll(f, -m, axis=axis) - np.roll(f, m - 1, axis=axis)) for m in (1, 2, 3)) / d


def cfl6(d, frac=0.9):
    """Largest stable step of the sixth-order leapfrog: |k~| is at most
    (2 / d_a) sum_m |c_m| per axis."""
    s = float(np.abs(C6).sum())
    return frac * 1.0 / (s * math.sqrt(sum(1.0 / v ** 2 for v in d)))


def test_coefficients_are_sixth_order():
    # the defining conditions, and the error of k~ shrinking 2^6 = 64 times per halving of k d
    assert abs(C6 @ [1, 3, 5] - 1) < 1e-14 and abs(C6 @ [1, 27, 125]) < 1e-13
    err = [abs(2 * _mod_sin(1.0, h) / h - 1.0) for h in (0.4, 0.2)]
    assert 60 < err[0] / err[1] < 68


@pytest.mark.parametrize("mode", [(3, 2), (1, 5), (7, 0)])
def test_sixth_order_2d_discrete_eigenmode(mode):
    n, d = (32, 24), (0.1, 0.13)
    dt = cfl6(d)
    kx, ky = 2 * math.pi * mode[0] / (n[0] * d[0]), 2 * math.pi * mode[1] / (n[1] * d[1])
    sx, sy = _mod_sin(kx, d[0]), _mod_sin(ky, d[1])
    s_w = dt * math.sqrt(sx ** 2 / d[0] ** 2 + sy ** 2 / d[1] ** 2)
    omega = 2 * math.asin(s_w) / dt
    i = np.arange(n[0])[None, :]
    j = np.arange(n[1])[:, None]
    bx = dt * sy / (d[1] * s_w)
    by = -dt * sx / (d[0] * s_w)

    def fields(t_e, t_b):
        Ez = np.cos(kx * i * d[0] + ky * j * d[1] - omega * t_e)
        Bx = bx * np.cos(kx * i * d[0] + ky * (j + 0.5) * d[1] - omega * t_b)
        By = by * np.cos(kx * (i + 0.5) * d[0] + ky * j * d[1] - omega * t_b)
        Bz = np.cos(kx * (i + 0.5) * d[0] + ky * (j + 0.5) * d[1] - omega * t_b)
        Ex = -bx * np.cos(kx * (i + 0.5) * d[0] + ky * j * d[1] - omega * t_e)
        Ey = -by * np.cos(kx * i * d[0] + ky * (j + 0.5) * d[1] - omega * t_e)
        return Ex, Ey, Ez, Bx, By, Bz

    def curl_e(Ex, Ey, Ez):
        return _dfw(Ez, 0, d[1]), -_dfw(Ez, 1, d[0]), _dfw(Ey, 1, d[0]) - _dfw(Ex, 0, d[1])

    Ex, Ey, Ez, Bx, By, Bz = fields(0.0, 0.5 * dt)
    cx, cy, cz = curl_e(Ex, Ey, Ez)
    grid = dict(ndim=2, n=list(n), d=list(d), dt=dt, patch=list(n), periodic=[1, 1], q=-1.0, m=1.0)
    s = oracle.Sim(grid)
    s.set_maxwell_order(6)
    for c, a in enumerate([Ex, Ey, Ez, Bx + 0.5 * dt * cx, By + 0.5 * dt * cy, Bz + 0.5 * dt * cz]):
        s.set_field(c, a)
    N = 300
    for _ in range(N):
        s.maxwell()
    ref = fields(N * dt, N * dt + 0.5 * dt)
    got = [s.field(c)[0] for c in range(6)]
    for a, b in zip(got[:3], ref[:3]):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-11)
    curl = curl_e(*got[:3])
    for a, b, c in zip(got[3:], ref[3:], curl):
        np.testing.assert_allclose(a - 0.5 * dt * c, b, rtol=0, atol=1e-11)


@pytest.mark.parametrize("mode", [(1, 2, 1), (3, 0, 2)])
def test_sixth_order_3d_discrete_eigenmode(mode):
    n, d = (16, 12, 10), (0.1, 0.13, 0.11)
    dt = cfl6(d)
    k = [2 * math.pi * mode[a] / (n[a] * d[a]) for a in range(3)]
    kt = np.array([2 * _mod_sin(k[a], d[a]) / d[a] for a in range(3)])
    s_w = 0.5 * dt * np.linalg.norm(kt)
    omega = 2 * math.asin(s_w) / dt
    e = np.cross(kt, [0.3, -0.7, 0.5])
    e /= np.linalg.norm(e)
    b = dt * np.cross(kt, e) / (2 * s_w)
    idx = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    pos = [idx[2], idx[1], idx[0]]

    def comp(c, amp, t):
        ph = sum(k[a] * (pos[a] + 0.5 * brute.STAG3[c][a]) * d[a] for a in range(3))
        return amp * np.cos(ph - omega * t)

    def fields(t_e, t_b):
        return [comp(c, e[c], t_e) for c in range(3)] + [comp(3 + c, b[c], t_b) for c in range(3)]

    def curl_e(E):
        dfw = lambda f, a: _dfw(f, 2 - a, d[a])
        return [dfw(E[2], 1) - dfw(E[1], 2), dfw(E[0], 2) - dfw(E[2], 0), dfw(E[1], 0) - dfw(E[0], 1)]

    F = fields(0.0, 0.5 * dt)
    curl = curl_e(F[:3])
    grid = dict(ndim=3, n=list(n), d=list(d), dt=dt, patch=list(n), periodic=[1, 1, 1], q=-1.0, m=1.0)
    s = oracle.Sim(grid)
    s.set_maxwell_order(6)
    for c in range(3):
        s.set_field(c, F[c])
        s.set_field(3 + c, F[3 + c] + 0.5 * dt * curl[c])
    N = 120
    for _ in range(N):
        s.maxwell()
    ref = fields(N * dt, N * dt + 0.5 * dt)
    got = [s.field(c) for c in range(6)]
    for c in range(3):
        np.testing.assert_allclose(got[c], ref[c], rtol=0, atol=1e-11)
    curl = curl_e(got[:3])
    for c in range(3):
        np.testing.assert_allclose(got[3 + c] - 0.5 * dt * curl[c], ref[3 + c], rtol=0, atol=1e-11)


def test_sixth_order_keeps_div_b():
    """B grows from random E; its sixth-order divergence (forward differences:
    Bx and By sit half a cell up along y and x) stays at rounding level."""
    n, d = (20, 16), (0.1, 0.12)
    dt = cfl6(d)
    g = np.random.default_rng(9)
    grid = dict(ndim=2, n=list(n), d=list(d), dt=dt, patch=list(n), periodic=[1, 1], q=-1.0, m=1.0)
    s = oracle.Sim(grid)
    s.set_maxwell_order(6)
    for c in range(3):
        s.set_field(c, g.standard_normal((n[1], n[0])))
    for _ in range(50):
        s.maxwell()
    Bx, By = s.field(3)[0], s.field(4)[0]
    div = _dfw(Bx, 1, d[0]) + _dfw(By, 0, d[1])
    assert np.abs(div).max() < 1e-11 * max(np.abs(Bx).max(), np.abs(By).max()) / min(d)


def test_sixth_order_needs_periodic_axes():
    grid = dict(ndim=2, n=[16, 8], d=[0.1, 0.1], dt=W.cfl_dt((0.1, 0.1)), patch=[16, 8],
                periodic=[0, 1], q=-1.0, m=1.0)
    s = oracle.Sim(grid)
    with pytest.raises(ValueError):
        s.set_maxwell_order(6)
    with pytest.raises(ValueError):
        oracle.Sim(dict(grid, periodic=[1, 1])).set_maxwell_order(4)
