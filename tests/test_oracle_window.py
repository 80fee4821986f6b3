"""Pins of the oracle's moving window (no GPU).

The window jumps one patch column when the distance it should have covered,
v c (n - start) dt after n steps, reaches the next multiple of the patch width.
With dyadic dt and cell size the jump steps are exact integers, so the
schedule is checked against integer arithmetic; the state right after a jump
must equal the state of the same run without a window, translated by one
patch column with numpy (fields with zeros entering, particles of the first
column dropped, every other patch renamed), plus the injected lattice built
here from its definition; and the injected plasma must carry exactly the
requested charge density (the quadratic shapes of a regular lattice sum to
one at every node).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle

Q = -1.0


def _grid(n=(32, 16), patch=(8, 8), d=(0.125, 0.125), dt=0.0625):
    return dict(ndim=2, n=list(n), d=list(d), dt=dt, patch=list(patch), periodic=[0, 1], q=Q, m=1.0)


def _empty(s):
    s.set_particles([np.zeros(0), np.zeros(0)], [np.zeros(0)] * 3, np.zeros(0))


@pytest.mark.parametrize("v,start,period", [(1.0, 5, 16), (0.5, 0, 32), (0.25, 3, 64)])
def test_jump_schedule_is_exact(v, start, period):
    # c dt / dx = 1/2 and 8-cell patches: one jump per 16 / v steps after `start`
    s = oracle.Sim(_grid())
    _empty(s)
    s.set_window(start, v, (1, 1), [0.0])
    seen = []
    for n in range(1, 3 * period + start + 2):
        s.step(1)
        seen.append(s.window_shift)
    want = [max(0, (n - start) // period) for n in range(1, 3 * period + start + 2)]
    assert seen == want


def _init(grid, seed):
    rng = np.random.default_rng(seed)
    n = grid["n"]
    k = 600
    x = [rng.uniform(0.5, n[0] - 0.5, k), rng.uniform(0, n[1], k)]
    u = [0.05 * rng.standard_normal(k) for _ in range(3)]
    w = rng.uniform(0.5, 1.5, k) * 1e-3
    F = [0.01 * rng.standard_normal((n[1], n[0] + 1)) for _ in range(6)]
    return x, u, w, F


def _make(grid, init, window=None):
    x, u, w, F = init
    s = oracle.Sim(grid)
    s.set_particles(x, u, w)
    for c, f in zip(("Ex", "Ey", "Ez", "Bx", "By", "Bz"), F):
        s.set_field(c, f)
    if window:
        s.set_window(*window)
    return s


def test_jump_is_a_translation_plus_injection():
    grid = _grid()
    init = _init(grid, 4)
    ppc = (2, 2)
    dens = np.array([0.01 * (c % 3) for c in range(64)])  # every third column empty
    A = _make(grid, init, (0, 1.0, ppc, dens))
    B = _make(grid, init)
    A.step(15)
    B.step(15)
    assert A.window_shift == 0
    for c in range(9):
        assert np.array_equal(A.field(c), B.field(c))
    A.step(1)
    B.step(1)
    assert A.window_shift == 1
    S, P1 = grid["patch"]
    npx, npy = grid["n"][0] // S, grid["n"][1] // P1
    # fields and currents: one patch column to the left, zeros entering
    for c in range(9):
        b = B.field(c)[0]
        want = np.zeros_like(b)
        want[:, :-S] = b[:, S:]
        assert np.array_equal(A.field(c)[0], want), c
    # particles: patch p takes patch p + 1's slots; the last column is injected
    bx, bu, bw, bid = B.particles()
    bc = B.counts()
    start = np.concatenate([[0], np.cumsum(bc)])
    n0 = bid.size + 0
    ex, ey, eu, ew, eid, ecount = [], [], [], [], [], []
    nxt = len(init[2])
    for py in range(npy):
        for px in range(npx):
            p = px + npx * py
            if px + 1 < npx:
                sl = slice(start[p + 1], start[p + 2])
                ex += list(bx[0][sl] - S)
                ey += list(bx[1][sl])
                eu += list(zip(bu[0][sl], bu[1][sl], bu[2][sl]))
                ew += list(bw[sl])
                eid += list(bid[sl])
                ecount.append(bc[p + 1])
            else:
                k0 = len(ex)
                for jl in range(P1):
                    for il in range(S):
                        col = S + (npx - 1) * S + il  # global column after the first jump
                        dn = dens[min(col, dens.size - 1)]
                        if dn <= 0:
                            continue
                        for b in range(ppc[1]):
                            for a in range(ppc[0]):
                                ex.append(px * S + il + (a + 0.5) / ppc[0])
                                ey.append(py * P1 + jl + (b + 0.5) / ppc[1])
                                eu.append((0.0, 0.0, 0.0))
                                ew.append(dn / (ppc[0] * ppc[1]))
                                eid.append(nxt)
                                nxt += 1
                ecount.append(len(ex) - k0)
    ax, au, aw, aid = A.particles()
    assert np.array_equal(A.counts(), np.array(ecount, dtype=np.int32))
    assert np.array_equal(aid, np.array(eid))
    assert np.array_equal(ax[0], np.array(ex)) and np.array_equal(ax[1], np.array(ey))
    assert np.array_equal(np.stack(au, 1), np.array(eu).reshape(-1, 3))
    assert np.array_equal(aw, np.array(ew))
    assert A.next_id == nxt
    assert A.removed == B.removed + int(sum(bc[npx * py] for py in range(npy)))
    assert n0 > 0 and A.counts()[npx - 1] > 0


def test_injected_plasma_has_the_table_density():
    grid = _grid()
    s = oracle.Sim(grid)
    _empty(s)
    dens = 0.02
    s.set_window(0, 1.0, (3, 2), [dens])
    s.step(16)
    assert s.window_shift == 1
    rho = s.rho()[0]
    n0 = grid["n"][0]
    # nodes whose four neighbouring cells all hold injected particles
    inner = rho[:, n0 - 6:n0 - 1]
    np.testing.assert_allclose(inner, Q * dens, rtol=1e-13, atol=0)
    assert np.all(rho[:, : n0 - 10] == 0.0)


def test_window_needs_an_open_x_axis_and_a_valid_speed():
    g = _grid()
    with pytest.raises(ValueError):
        oracle.Sim(dict(g, periodic=[1, 1])).set_window(0, 1.0, (1, 1), [0.0])
    for v in (0.0, 1.5, -1.0):
        with pytest.raises(ValueError):
            oracle.Sim(g).set_window(0, v, (1, 1), [0.0])
    with pytest.raises(ValueError):
        oracle.Sim(g).set_window(0, 1.0, (0, 1), [0.0])
    with pytest.raises(ValueError):
        oracle.Sim(g).set_window(0, 1.0, (1, 1), [-1.0])
