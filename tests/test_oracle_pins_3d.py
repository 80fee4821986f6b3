"""Pins of the FP64 oracle in three dimensions (no GPU).

Brute-force gather over every node and periodic image, Esirkepov currents
against quadrature of the defining time integral, continuity and the
total-current identity, a discrete 3-D Yee eigenmode at the frequency of the
Yee dispersion relation, div B = 0 and the Gauss law under the full loop, and
re-binning invariants with 26 neighbour directions.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from tests import fixtures as W
from tests import brute


def grid3(n=(6, 6, 6), d=(0.1, 0.12, 0.09), patch=None, dt=None):
    patch = patch or n
    return dict(ndim=3, n=list(n), d=list(d), dt=dt or W.cfl_dt(d), patch=list(patch),
                periodic=[1, 1, 1], q=-1.0, m=1.0)


def test_gather_3d_matches_all_node_sum_with_images():
    n = (6, 5, 7)
    g = np.random.default_rng(31)
    s = oracle.Sim(grid3(n))
    fields = [g.standard_normal((n[2], n[1], n[0])) for _ in range(6)]
    for c, f in enumerate(fields):
        s.set_field(c, f)
    for _ in range(25):
        xi = g.uniform(0, 1, 3) * np.array(n)
        got = s.gather(xi)
        ref = brute.gather_3d(fields, xi, n)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_gather_3d_reproduces_linear_field():
    # a field linear along x (periodic only in its constant part): on nodes far
    # from the seam the quadratic spline reproduces it exactly
    n = (12, 6, 6)
    s = oracle.Sim(grid3(n))
    xnode = np.arange(n[0], dtype=float)
    for c in range(6):
        st = brute.STAG3[c][0]
        f = np.broadcast_to(2.0 + 0.25 * (xnode + 0.5 * st), (n[2], n[1], n[0]))
        s.set_field(c, np.ascontiguousarray(f))
    for xi in ([5.3, 2.2, 4.9], [6.1, 0.4, 3.3], [4.75, 5.5, 1.0]):
        got = s.gather(xi)
        np.testing.assert_allclose(got, 2.0 + 0.25 * xi[0], rtol=0, atol=1e-13)


def _currents_3d(x0, x1, w=0.7, n=(10, 10, 10), d=(0.1, 0.12, 0.09), dt=0.04):
    s = oracle.Sim(grid3(n, d=d, dt=dt))
    s.deposit(x0, x1, w, 0.0)
    return [s.field(c) for c in ("Jx", "Jy", "Jz")]


def test_esirkepov_3d_matches_time_integral_quadrature():
    g = np.random.default_rng(32)
    n, d, dt = (10, 10, 10), (0.1, 0.12, 0.09), 0.04
    for _ in range(25):
        x0 = g.uniform(3, 7, 3)
        x1 = x0 + g.uniform(-0.99, 0.99, 3)
        J = _currents_3d(x0, x1, n=n, d=d, dt=dt)
        ref = brute.esirkepov_quadrature_3d(x0, x1, 0.7, -1.0, d, dt, n)
        for a in range(3):
            np.testing.assert_allclose(J[a], ref[a], rtol=0, atol=1e-13 * max(1, np.abs(ref[a]).max()))


def test_esirkepov_3d_continuity_and_total_current():
    g = np.random.default_rng(33)
    n, d, dt = (8, 8, 8), (0.1, 0.12, 0.09), 0.04
    for _ in range(20):
        x0 = g.uniform(0, 8, 3)
        x1 = x0 + g.uniform(-0.99, 0.99, 3)  # may cross periodic seams
        J = _currents_3d(x0, x1, n=n, d=d, dt=dt)
        r0 = brute.rho_3d([[x0[0]], [x0[1]], [x0[2]]], [0.7], -1.0, n)
        r1 = brute.rho_3d([[x1[0] % 8], [x1[1] % 8], [x1[2] % 8]], [0.7], -1.0, n)
        res = (r1 - r0) / dt + brute.div_dual_3d(J, d)
        assert np.abs(res).max() < 1e-12 * np.abs(r0).max() / dt
        for a in range(3):
            assert abs(J[a].sum() - (-1.0) * 0.7 * d[a] * (x1[a] - x0[a]) / dt) < 1e-12


def test_esirkepov_3d_stationary_particle_deposits_nothing():
    J = _currents_3d([4.3, 5.1, 2.7], [4.3, 5.1, 2.7])
    assert all(np.all(j == 0.0) for j in J)


def _curl_e_3d(E, d):
    """Forward-difference curl of E onto the B positions (periodic)."""
    def dfw(f, a):
        return (np.roll(f, -1, axis=2 - a) - f) / d[a]
    return [dfw(E[2], 1) - dfw(E[1], 2), dfw(E[0], 2) - dfw(E[2], 0), dfw(E[1], 0) - dfw(E[0], 1)]


@pytest.mark.parametrize("mode", [(1, 2, 1), (3, 0, 2)])
def test_yee_3d_discrete_eigenmode(mode):
    """A discrete 3-D plane wave (polarisation normal to the discrete wave
    vector kt_a = 2 sin(k_a d_a / 2) / d_a) evolves exactly at the frequency
    of sin(w dt / 2) = (dt / 2) |kt|."""
    n, d = (16, 12, 10), (0.1, 0.13, 0.11)
    dt = W.cfl_dt(d, 0.95)
    k = [2 * math.pi * mode[a] / (n[a] * d[a]) for a in range(3)]
    kt = np.array([2 * math.sin(k[a] * d[a] / 2) / d[a] for a in range(3)])
    s_w = 0.5 * dt * np.linalg.norm(kt)
    omega = 2 * math.asin(s_w) / dt
    e = np.cross(kt, [0.3, -0.7, 0.5])
    e /= np.linalg.norm(e)
    b = dt * np.cross(kt, e) / (2 * s_w)
    idx = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    pos = [idx[2], idx[1], idx[0]]  # x, y, z node indices as (nz, ny, nx) arrays

    def comp(c, amp, t):
        ph = sum(k[a] * (pos[a] + 0.5 * brute.STAG3[c][a]) * d[a] for a in range(3))
        return amp * np.cos(ph - omega * t)

    def fields(t_e, t_b):
        return [comp(c, e[c], t_e) for c in range(3)] + [comp(3 + c, b[c], t_b) for c in range(3)]

    F = fields(0.0, 0.5 * dt)
    curl = _curl_e_3d(F[:3], d)
    s = oracle.Sim(grid3(n, d=d, dt=dt))
    for c in range(3):
        s.set_field(c, F[c])
        s.set_field(3 + c, F[3 + c] + 0.5 * dt * curl[c])
    N = 150
    for _ in range(N):
        s.maxwell()
    ref = fields(N * dt, N * dt + 0.5 * dt)
    got = [s.field(c) for c in range(6)]
    for c in range(3):
        np.testing.assert_allclose(got[c], ref[c], rtol=0, atol=1e-11)
    curl = _curl_e_3d(got[:3], d)
    for c in range(3):
        np.testing.assert_allclose(got[3 + c] - 0.5 * dt * curl[c], ref[3 + c], rtol=0, atol=1e-11)


def _small_blob(n=(16, 16, 8), patch=(8, 8, 4), T_keV=20.0):
    return W.blob_3d(n=n, d=(0.1, 0.1, 0.1), patch=patch, ppc0=2, blob_radius=3.0, T_keV=T_keV)


def test_yee_3d_div_b_and_gauss_law_with_deposit():
    wl = _small_blob()
    s = oracle.Sim(wl["grid"])
    s.set_particles(wl["x"], wl["u"], wl["w"])
    d = wl["grid"]["d"]
    rho0 = s.rho()
    for _ in range(8):
        s.step(1)
    E = [s.field(c) for c in ("Ex", "Ey", "Ez")]
    B = [s.field(c) for c in ("Bx", "By", "Bz")]
    divE = sum((E[a] - np.roll(E[a], 1, axis=2 - a)) / d[a] for a in range(3))
    rho = s.rho() - rho0
    assert np.abs(divE - rho).max() < 1e-11 * np.abs(rho0).max()
    divB = sum((np.roll(B[a], -1, axis=2 - a) - B[a]) / d[a] for a in range(3))
    assert np.abs(divB).max() < 1e-11


def test_rebin_3d_invariants_over_the_loop():
    """26 neighbour directions: every particle sits in its own patch, ids stay
    a permutation, counts add up, and particles that stay keep their order."""
    wl = _small_blob(T_keV=200.0)  # hot: many patch crossings per step
    s = oracle.Sim(wl["grid"])
    s.set_particles(wl["x"], wl["u"], wl["w"])
    npart = wl["w"].size
    P = wl["grid"]["patch"]
    npx = [wl["grid"]["n"][a] // P[a] for a in range(3)]
    for _ in range(6):
        x0, _, _, id0 = s.particles()
        c0 = s.counts()
        s.step(1)
        x, _, _, ids = s.particles()
        c = s.counts()
        assert c.sum() == npart and np.array_equal(np.sort(ids), np.arange(npart))
        pid = np.repeat(np.arange(c.size), c)
        cell = [np.floor(x[a]).astype(np.int64) // P[a] for a in range(3)]
        assert np.array_equal(pid, cell[0] + npx[0] * (cell[1] + npx[1] * cell[2]))
        # stayers below the new count that were not vacated keep their slots
        off0 = np.concatenate([[0], np.cumsum(c0)])
        off1 = np.concatenate([[0], np.cumsum(c)])
        moved = 0
        for p in range(c.size):
            a, b = id0[off0[p]:off0[p + 1]], ids[off1[p]:off1[p + 1]]
            m = min(a.size, b.size)
            same = a[:m] == b[:m]
            moved += int((~same).sum())
        assert moved < npart // 4
