"""The oracle's particle merging against a brute-force reference (no GPU).

`tests/brute.py` restates the clustering (weighted Lloyd iterations in
momentum, centroids started at members floor(j n / k), nearest centroid with
the lowest index on ties, weighted-mean updates that leave empty clusters
where they are) with numpy distance matrices and argmin, and the conserving
pair of a cluster from its totals.  A merge pass of the oracle over one
crowded cell must keep exactly the particles of the clusters with fewer than
three members, in slot order, and append one pair per larger cluster, in
cluster order.  An unweighted or unordered centroid update, another start,
a missed round or a wrong tie rule changes which particles are kept or the
pair momenta.  The reference's own centroid history is checked against
Lloyd's property that no round raises the weighted within-cluster sum of
squares.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests.brute import lloyd_cell, merge_pair

CELL = (3, 5)


def _grid():
    return dict(ndim=2, n=[8, 8], d=[0.1, 0.1], dt=0.05, patch=[8, 8], periodic=[1, 1], q=-1.0, m=1.0)


def _state(rng, n, cmax, umom, wts):
    """n particles in CELL (momenta umom, weights wts) interleaved with
    particles of uncrowded cells (at most cmax each)."""
    xs, ys, us, ws, crowded = [], [], [], [], []
    others = [(0, 0), (6, 2), (3, 4), (7, 7)]
    k_other = [int(rng.integers(0, cmax + 1)) for _ in others]
    order = [("c", i) for i in range(n)] + [("o", j) for j, c in enumerate(k_other) for _ in range(c)]
    perm = rng.permutation(len(order))
    for pos in perm:
        kind, i = order[pos]
        if kind == "c":
            cx, cy = CELL
            crowded.append(len(ws))
            us.append(umom[i])
            ws.append(wts[i])
        else:
            cx, cy = others[i]
            us.append(rng.standard_normal(3))
            ws.append(rng.uniform(0.5, 1.5))
        xs.append(cx + rng.uniform(0.0, 1.0))
        ys.append(cy + rng.uniform(0.0, 1.0))
    u = np.array(us)
    return [np.array(xs), np.array(ys)], [u[:, 0], u[:, 1], u[:, 2]], np.array(ws), np.array(crowded)


def _expected(x, u, w, crowded, cmax, iters):
    U = np.stack(u, axis=1)
    X = np.stack(x, axis=1)
    ids = np.arange(w.size)
    k = cmax // 2
    asg, hist = lloyd_cell(U[crowded], w[crowded], k, iters)
    keep = np.ones(w.size, dtype=bool)
    pairs = []
    for j in range(k):
        mem = crowded[asg == j]
        if mem.size >= 3:
            keep[mem] = False
            pairs += merge_pair(U[mem], w[mem], X[mem], ids[mem])
    return keep, pairs, asg, hist


def _sse(U, w, asg, cen):
    return float(sum(w[i] * np.sum((U[i] - cen[asg[i]]) ** 2) for i in range(w.size)))


def _check(x, u, w, crowded, cmax, iters):
    s = oracle.Sim(_grid())
    s.set_particles(x, u, w)
    taken = s.merge(cmax, iters)
    ox, ou, ow, oid = s.particles()
    keep, pairs, asg, hist = _expected(x, u, w, crowded, cmax, iters)
    nk = int(keep.sum())
    assert taken == w.size - nk - len(pairs)
    assert np.array_equal(oid[:nk], np.flatnonzero(keep))
    assert np.array_equal(ow[:nk], w[keep])
    for t, (X, P, W, pid) in enumerate(pairs):
        q = nk + t
        assert oid[q] == pid
        assert ow[q] == pytest.approx(W, rel=1e-14)
        np.testing.assert_allclose([ox[0][q], ox[1][q]], X, rtol=1e-14, atol=1e-14)
        np.testing.assert_allclose([ou[0][q], ou[1][q], ou[2][q]], P, rtol=1e-12, atol=1e-12)
    # Lloyd: no round raises the weighted within-cluster sum of squares
    U = np.stack(u, axis=1)[crowded]
    ww = w[crowded]
    k = cmax // 2
    cen = np.array([U[(j * len(ww)) // k] for j in range(k)])
    prev = None
    for c in hist:
        d2 = ((U[:, None, :] - cen[None, :, :]) ** 2).sum(axis=2)
        a = np.argmin(d2, axis=1)
        e = _sse(U, ww, a, c)
        if prev is not None:
            assert e <= prev * (1 + 1e-12) + 1e-300
        prev = e
        cen = c
    return asg


@pytest.mark.parametrize("n,cmax,iters,seed", [(5, 4, 1, 1), (9, 8, 3, 2), (17, 16, 8, 3),
                                               (25, 16, 2, 4), (40, 32, 10, 5), (40, 8, 20, 6),
                                               (33, 32, 64, 7)])
def test_merge_of_a_crowded_cell_matches_brute_force(n, cmax, iters, seed):
    rng = np.random.default_rng(seed)
    umom = rng.standard_normal((n, 3)) * rng.uniform(0.1, 4.0)
    wts = rng.uniform(0.1, 3.0, n)
    x, u, w, crowded = _state(rng, n, cmax, umom, wts)
    _check(x, u, w, crowded, cmax, iters)


def test_ties_and_empty_clusters():
    """Duplicated momenta: starting centroids coincide (the later ones never
    win a tie and stay empty) and members at equal distance go to the lowest
    index."""
    rng = np.random.default_rng(11)
    n, cmax = 12, 8
    base = np.array([[0.5, 0.0, 0.0], [-0.5, 0.2, 0.1], [2.0, -1.0, 0.3]])
    umom = base[np.arange(n) % 3]
    wts = rng.uniform(0.5, 2.0, n)
    x, u, w, crowded = _state(rng, n, cmax, umom, wts)
    asg = _check(x, u, w, crowded, cmax, 5)
    assert len(set(asg.tolist())) <= 3


def test_weights_decide_the_clusters():
    """Cells with widely spread weights: the oracle follows the weighted
    reference on every one, and on some of them an unweighted update would
    have ended with another partition (so the check sees the weights)."""
    differ = 0
    for seed in range(20, 40):
        rng = np.random.default_rng(seed)
        n, cmax = 14, 4
        umom = rng.standard_normal((n, 3))
        wts = np.exp(rng.uniform(-4.0, 4.0, n))
        x, u, w, crowded = _state(rng, n, cmax, umom, wts)
        _check(x, u, w, crowded, cmax, 6)
        U = np.stack(u, axis=1)[crowded]
        a_w, _ = lloyd_cell(U, w[crowded], cmax // 2, 6)
        a_1, _ = lloyd_cell(U, np.ones(len(crowded)), cmax // 2, 6)
        differ += not np.array_equal(a_w, a_1)
    assert differ >= 3
