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
