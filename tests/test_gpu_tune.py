"""The patch-size tuner (pic_autotune_patch): it times temporary simulations
at each candidate patch edge and workgroup size, writes the fastest into the
descriptor, reuses a cached choice, and the tuned descriptor runs the same
physics as the oracle with that patch."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1511_03878_amd import workloads as W
from paper_1511_03878_amd.sim import autotune_patch
from tests.helpers import compare_fields, gpu_sim, oracle_run

pytestmark = pytest.mark.gpu


def test_patch_tuner(tmp_path):
    print("[gpu-test] pic_autotune_patch on the small laser box", flush=True)
    wl = W.lwfa_2d_small()
    cache = str(tmp_path / "tune.txt")
    grid, tune, r = autotune_patch(wl, 32, candidates=(8, 16, 32, 24), warm=5, steps=5, cache=cache)
    assert grid["patch"][0] == grid["patch"][1] in (8, 16, 32)
    assert tune["block"] in (256, 512, 1024)
    assert r["from_cache"] == 0 and r["trials"] >= 3 and r["ms_per_step"] > 0
    assert r["patch"][:2] == grid["patch"]
    grid2, tune2, r2 = autotune_patch(wl, 32, candidates=(8, 16, 32, 24), warm=5, steps=5, cache=cache)
    assert r2["from_cache"] == 1 and grid2 == grid and tune2 == tune
    tuned = dict(wl, grid=grid)
    g = gpu_sim(tuned, 64, **tune)
    g.step(20)
    o = oracle_run(tuned, 20)
    e, b = compare_fields(g, o)
    assert e < 1e-11 and b < 1e-11, (e, b)
    assert np.array_equal(g.counts(), o.counts())
