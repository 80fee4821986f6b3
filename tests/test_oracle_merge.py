"""Pins of the oracle's particle merging (no GPU).

What the merge must keep is fixed by the physics, not by the oracle: in every
cell the total weight (charge), momentum, kinetic energy and first moment of
the charge stay as they were; cells at or below the threshold are untouched;
after a pass no cell holds more than cmax particles; identical particles merge
into copies of themselves; well-separated momentum groups end in separate
pairs, each carrying its group's two smallest ids.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle


def _grid(n=(16, 16), patch=(8, 8)):
    return dict(ndim=2, n=list(n), d=[0.1, 0.1], dt=0.05, patch=list(patch), periodic=[1, 1], q=-1.0, m=1.0)


def _cells(x, y):
    return np.floor(x).astype(int) + 1000 * np.floor(y).astype(int)


def _moments(x, u, w):
    """Per cell: weight, momentum, kinetic energy, first moment of weight."""
    g = np.sqrt(1.0 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    cells = _cells(x[0], x[1])
    out = {}
    for c in np.unique(cells):
        m = cells == c
        out[c] = np.array([w[m].sum(), (w[m] * u[0][m]).sum(), (w[m] * u[1][m]).sum(), (w[m] * u[2][m]).sum(),
                           (w[m] * (g[m] - 1.0)).sum(), (w[m] * x[0][m]).sum(), (w[m] * x[1][m]).sum()])
    return out, cells


def _dense_state(seed, n=(16, 16), per_cell=None, umax=5.0):
    rng = np.random.default_rng(seed)
    if per_cell is None:
        per_cell = rng.integers(0, 60, size=n[0] * n[1])
    xs, ys = [], []
    for c, k in enumerate(per_cell):
        cx, cy = c % n[0], c // n[0]
        xs.append(cx + rng.uniform(0, 1, k))
        ys.append(cy + rng.uniform(0, 1, k))
    x = [np.concatenate(xs), np.concatenate(ys)]
    N = x[0].size
    u = [umax * rng.standard_normal(N) for _ in range(3)]
    w = rng.uniform(0.2, 2.0, N)
    return x, u, w


@pytest.mark.parametrize("cmax,iters,seed", [(16, 8, 1), (4, 3, 2), (32, 20, 3)])
def test_merge_keeps_every_cells_conserved_quantities(cmax, iters, seed):
    x, u, w = _dense_state(seed)
    s = oracle.Sim(_grid())
    s.set_particles(x, u, w)
    bx, bu, bw, bid = s.particles()
    before, bcells = _moments(bx, bu, bw)
    taken = s.merge(cmax, iters)
    ax, au, aw, aid = s.particles()
    after, acells = _moments(ax, au, aw)
    assert taken == bw.size - aw.size > 0 and s.merged == taken
    assert set(after) == set(before)
    for c in before:
        np.testing.assert_allclose(after[c], before[c], rtol=1e-12, atol=1e-12)
        assert np.count_nonzero(acells == c) <= max(cmax, np.count_nonzero(bcells == c))
        assert np.count_nonzero(acells == c) <= cmax or np.count_nonzero(bcells == c) <= cmax
    # cells at or below the threshold: the same particles, bit for bit
    for c in before:
        if np.count_nonzero(bcells == c) <= cmax:
            mb, ma = bcells == c, acells == c
            assert np.array_equal(np.sort(bid[mb]), np.sort(aid[ma]))
    # ids stay unique and come from the original set
    assert np.unique(aid).size == aid.size and np.isin(aid, bid).all()
    # a second pass finds nothing to do
    assert s.merge(cmax, iters) == 0


def test_identical_particles_merge_into_copies():
    n = 40
    x = [np.full(n, 3.25), np.full(n, 5.5)]
    u = [np.full(n, 0.3), np.full(n, -2.0), np.full(n, 1.25)]
    w = np.full(n, 0.5)
    s = oracle.Sim(_grid())
    s.set_particles(x, u, w)
    s.merge(4, 5)  # k = 2: both centroids start on the same point, one cluster takes all
    ax, au, aw, aid = s.particles()
    assert aw.size == 2
    np.testing.assert_allclose(aw, [10.0, 10.0], rtol=1e-14)
    for a, v in enumerate((0.3, -2.0, 1.25)):
        np.testing.assert_allclose(au[a], [v, v], rtol=1e-12)
    assert sorted(aid) == [0, 1]


def test_separated_groups_end_in_separate_pairs():
    rng = np.random.default_rng(4)
    n = 30
    x = [3.0 + rng.uniform(0, 1, n), 2.0 + rng.uniform(0, 1, n)]
    grp = np.arange(n) % 2  # interleaved: member 0 in group 0, member n/2 = 15 in group 1
    cen = np.array([[4.0, 0.0, 0.0], [-1.0, 3.0, 0.5]])
    u = [cen[grp, a] + 1e-3 * rng.standard_normal(n) for a in range(3)]
    w = rng.uniform(0.5, 1.5, n)
    s = oracle.Sim(_grid())
    s.set_particles(x, u, w)
    s.merge(4, 6)
    ax, au, aw, aid = s.particles()
    assert aw.size == 4
    ids = np.arange(n)
    for gi in range(2):
        m = grp == gi
        P = np.array([(w[m] * u[a][m]).sum() for a in range(3)])
        pair = np.isin(aid, np.sort(ids[m])[:2])
        assert pair.sum() == 2
        np.testing.assert_allclose(aw[pair].sum(), w[m].sum(), rtol=1e-13)
        np.testing.assert_allclose([(aw[pair] * au[a][pair]).sum() for a in range(3)], P, rtol=1e-12, atol=1e-12)


def test_merge_after_steps_and_refusals():
    x, u, w = _dense_state(7, per_cell=np.full(256, 20))
    g = _grid()
    s = oracle.Sim(g)
    s.set_particles(x, [0.01 * v for v in u], w)
    s.set_merge(3, 16, 4)
    s.step(2)
    assert s.merged == 0
    s.step(1)
    assert s.merged > 0
    _, cnt = np.unique(_cells(*s.particles()[0][:2]), return_counts=True)
    assert cnt.max() <= 16
    with pytest.raises(ValueError):
        s.set_merge(1, 2, 4)
    with pytest.raises(ValueError):
        s.set_merge(1, 40, 4)
    with pytest.raises(ValueError):
        s.merge(16, 0)
