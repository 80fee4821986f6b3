"""Pins of the Hilbert-curve patch order and the cost-balanced segments
(oracle, no GPU): the end points the paper gives for its 32 x 32 example,
one visit per patch with unit steps, the recursive block structure that
makes curve segments compact, and the load bound of the segment rule against
brute-force optimal partitions of small inputs."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from oracle import hilbert as H


def _coords(order, np_):
    if len(np_) == 2:
        return [(p % np_[0], p // np_[0]) for p in order]
    nx, ny = np_[0], np_[1]
    return [(p % nx, (p // nx) % ny, p // (nx * ny)) for p in order]


def _unit_steps(pts):
    return all(sum(abs(a[i] - b[i]) for i in range(len(a))) == 1 for a, b in zip(pts, pts[1:]))


def test_paper_example_32x32_endpoints_and_single_visits():
    order = H.patch_order((32, 32))
    pts = _coords(order, (32, 32))
    assert sorted(order) == list(range(1024))
    assert pts[0] == (0, 0) and pts[-1] == (31, 0)
    assert _unit_steps(pts)


@pytest.mark.parametrize("side", [1, 2, 4, 8, 16, 64])
def test_square_curves(side):
    pts = [H.square_point(side, d) for d in range(side * side)]
    assert len(set(pts)) == side * side and all(0 <= x < side and 0 <= y < side for x, y in pts)
    assert pts[0] == (0, 0) and pts[-1] == (side - 1, 0)
    assert _unit_steps(pts)


@pytest.mark.parametrize("side", [2, 4, 8, 16])
def test_square_curve_blocks_are_aligned_squares(side):
    """Positions [k 4^m, (k + 1) 4^m) cover exactly one aligned 2^m x 2^m block."""
    pts = [H.square_point(side, d) for d in range(side * side)]
    m = 1
    while (1 << m) <= side:
        b = 1 << m
        for k in range(side * side // (b * b)):
            blk = pts[k * b * b:(k + 1) * b * b]
            x0, y0 = min(p[0] for p in blk), min(p[1] for p in blk)
            assert x0 % b == 0 and y0 % b == 0
            assert set(blk) == {(x0 + i, y0 + j) for i in range(b) for j in range(b)}
        m += 1


@pytest.mark.parametrize("np_", [(128, 32), (32, 128), (16, 2), (2, 16), (8, 8), (4, 1), (1, 4)])
def test_rectangular_2d_orders(np_):
    order = H.patch_order(np_)
    pts = _coords(order, np_)
    assert sorted(order) == list(range(np_[0] * np_[1]))
    assert pts[0] == (0, 0)
    assert _unit_steps(pts)


@pytest.mark.parametrize("side", [2, 4, 8])
def test_cube_curves(side):
    pts = [H.cube_point(side, d) for d in range(side ** 3)]
    assert len(set(pts)) == side ** 3
    assert pts[0] == (0, 0, 0) and pts[-1] == (side - 1, 0, 0)
    assert _unit_steps(pts)
    # positions [k 8^m, (k + 1) 8^m) cover one aligned 2^m cube
    for m in range(1, side.bit_length()):
        b = 1 << m
        for k in range(side ** 3 // b ** 3):
            blk = pts[k * b ** 3:(k + 1) * b ** 3]
            lo = [min(p[a] for p in blk) for a in range(3)]
            assert all(v % b == 0 for v in lo)
            assert set(blk) == set(itertools.product(*[range(lo[a], lo[a] + b) for a in range(3)]))


@pytest.mark.parametrize("np_", [(8, 4, 4), (4, 8, 4), (4, 4, 8), (2, 2, 2), (64, 32, 32)])
def test_3d_orders(np_):
    order = H.patch_order(np_)
    pts = _coords(order, np_)
    assert sorted(order) == list(range(int(np.prod(np_))))
    assert pts[0] == (0, 0, 0)
    assert _unit_steps(pts)


def test_unsupported_grids_raise():
    with pytest.raises(ValueError):
        H.patch_order((12, 8))
    with pytest.raises(ValueError):
        H.patch_order((8, 4, 2))


def _best_bottleneck(costs, k):
    n = len(costs)
    best = None
    for cuts in itertools.combinations_with_replacement(range(n + 1), k - 1):
        b = (0,) + cuts + (n,)
        if any(b[i] > b[i + 1] for i in range(k)):
            continue
        worst = max(sum(costs[b[i]:b[i + 1]]) for i in range(k))
        best = worst if best is None else min(best, worst)
    return best


def test_segments_bound_and_brute_force():
    g = np.random.default_rng(5)
    for _ in range(60):
        n = int(g.integers(1, 9))
        k = int(g.integers(1, 5))
        costs = [int(v) for v in g.integers(0, 50, n)]
        b = H.segments(costs, k)
        assert len(b) == k + 1 and b[0] == 0 and b[-1] == n
        assert all(b[i] <= b[i + 1] for i in range(k))
        seg = [sum(costs[b[i]:b[i + 1]]) for i in range(k)]
        total, cmax = sum(costs), max(costs)
        assert max(seg) * k <= total + k * cmax
        best = _best_bottleneck(costs, k)
        assert best <= max(seg) <= best + cmax


def test_segments_of_the_paper_example_are_compact():
    """Seven equal-count segments of the 32 x 32 curve (the paper's Fig. 2
    example): each is a connected set of patches, and together they have a
    shorter interface than seven row-major strips of the same sizes."""
    order = H.patch_order((32, 32))
    b = H.segments([1] * 1024, 7)
    owner_h = np.empty(1024, dtype=int)
    owner_r = np.empty(1024, dtype=int)
    for j in range(7):
        owner_h[order[b[j]:b[j + 1]]] = j
        owner_r[b[j]:b[j + 1]] = j

    def interface(owner):
        o = owner.reshape(32, 32)
        return int((o[:, 1:] != o[:, :-1]).sum() + (o[1:, :] != o[:-1, :]).sum())

    assert interface(owner_h) < interface(owner_r)
    for j in range(7):
        pts = _coords(order[b[j]:b[j + 1]], (32, 32))
        assert _unit_steps(pts)
