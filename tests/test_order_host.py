"""The C-ABI patch order and curve segments (host logic, no GPU) against the
oracle: exact integer agreement on square, rectangular and 3-D patch grids,
and the documented errors."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import hilbert as H
from paper_1511_03878_amd import sim
from paper_1511_03878_amd._capi import PicError


@pytest.mark.parametrize("np_", [(32, 32), (128, 32), (32, 128), (16, 4), (1, 8), (8, 1), (1, 1),
                                 (8, 4, 4), (4, 8, 4), (4, 4, 8), (64, 32, 32), (2, 2, 2)])
def test_patch_order_matches_oracle(np_):
    assert np.array_equal(sim.patch_order(np_), np.array(H.patch_order(np_), dtype=np.int32))


def test_curve_segments_match_oracle():
    g = np.random.default_rng(2)
    for _ in range(300):
        n = int(g.integers(0, 70))
        k = int(g.integers(1, 12))
        c = g.integers(0, 10 ** 9, n)
        got = sim.curve_segments(c, k)
        assert np.array_equal(got, np.array(H.segments([int(v) for v in c], k)))


def test_order_errors():
    with pytest.raises(PicError) as e:
        sim.patch_order((12, 8))
    assert e.value.code == -9  # PIC_ENOTSUP
    with pytest.raises(PicError):
        sim.patch_order((8, 4, 2))
    with pytest.raises(PicError) as e:
        sim.curve_segments([1, -1, 2], 2)
    assert e.value.code == -1
    with pytest.raises(PicError):
        sim.curve_segments([1, 2], 0)


def _blocks_contiguous(pts, nd, b):
    """Every aligned block of side b holds consecutive curve positions."""
    seen = {}
    for i, p in enumerate(pts):
        key = tuple(v // b for v in p)
        seen.setdefault(key, []).append(i)
    return all(v[-1] - v[0] + 1 == len(v) for v in seen.values())


@pytest.mark.parametrize("np_", [(2, 2, 2), (4, 4, 4), (8, 8, 8), (16, 16, 16), (16, 8, 8), (8, 32, 8),
                                 (32, 16, 16)])
def test_patch_order_3d_is_a_hilbert_order(np_):
    """The product's 3-D order pinned by the defining properties of a
    Hilbert-type curve, independently of the oracle (3-D Hilbert curves are
    not unique; both sides use the published transpose routine): every patch
    once, face-neighbour steps, each aligned cube of side 2^m visited as one
    contiguous run at every level m, start at the origin, and each cube of
    the shortest side (a square's side in the paper's 2-D figure) left at its
    far corner along the longest axis."""
    order = sim.patch_order(np_)
    nx, ny = np_[0], np_[1]
    pts = [(int(p) % nx, (int(p) // nx) % ny, int(p) // (nx * ny)) for p in order]
    assert sorted(order.tolist()) == list(range(int(np.prod(np_))))
    assert all(sum(abs(a[i] - b[i]) for i in range(3)) == 1 for a, b in zip(pts, pts[1:]))
    side = min(np_)
    m = 1
    while (1 << m) <= side:
        assert _blocks_contiguous(pts, 3, 1 << m), (np_, 1 << m)
        m += 1
    assert pts[0] == (0, 0, 0)
    long_ax = int(np.argmax(np_))
    cubes = int(np.prod(np_)) // side ** 3
    if cubes == 1:
        end = [0, 0, 0]
        end[0] = side - 1
        assert pts[-1] == tuple(end)
    else:
        assert pts[-1][long_ax] == np_[long_ax] - 1
