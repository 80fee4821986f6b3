"""Parity of the HIP path (through the C ABI) with the FP64 oracle on MI355X.

Tolerances: FP64 fields within 1e-11 relative L2 after 10 steps; FP32 within
1e-5 after one step; patch occupancy and the slot of every particle (its id)
bit-exact.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests import fixtures as W
from tests.helpers import compare_fields, gpu_sim, neighbour_patch, oracle_run, rel_l2

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def c1():
    return W.uniform_2d()


def test_uniform_fp64_ten_steps_match_oracle(c1):
    _announce("uniform 128x128 16ppc fp64, 10 steps")
    g = gpu_sim(c1, 64)
    g.step(10)
    o = oracle_run(c1, 10)
    e, b = compare_fields(g, o)
    assert e < 1e-11 and b < 1e-11, (e, b)
    assert np.array_equal(g.counts(), o.counts())
    gx, gu, gw, gid = g.particles()
    ox, ou, ow, oid = o.particles()
    assert np.array_equal(gid, oid)
    for a in range(2):
        assert np.abs(gx[a] - ox[a]).max() < 1e-11
    for a in range(3):
        assert np.abs(gu[a] - ou[a]).max() < 1e-12
    d = g.diag()
    assert d["step"] == 10 and d["particles"] == c1["w"].size
    # energies of the last step: field energy of E^9, B^9 and K^9
    U, K, pushed = g.history(9, 1)
    Uo, Ko = o.energy()
    assert abs(U[0] - Uo) <= 1e-10 * abs(Uo) and abs(K[0] - Ko) <= 1e-12 * abs(Ko)
    assert pushed[0] == c1["w"].size


def test_uniform_fp32_one_step_matches_oracle(c1):
    _announce("uniform 128x128 16ppc fp32, 1 step")
    wl = W.to_float32_state(c1)
    g = gpu_sim(wl, 32)
    g.step(1)
    o = oracle_run(wl, 1)
    e, b = compare_fields(g, o)
    assert e < 1e-5 and b < 1e-5, (e, b)
    assert np.array_equal(g.counts(), o.counts())
    jg = [g.field(c) for c in ("Jx", "Jy", "Jz")]
    jo = [o.field(c)[0] for c in ("Jx", "Jy", "Jz")]
    assert rel_l2(jg, jo) < 1e-5


def test_box_of_16384_patches_matches_oracle_fp64():
    # more patches than the one-workgroup queue build caches (8192): the
    # work queue comes from the grid-wide histogram and placement kernels
    _announce("uniform 512x512, 4x4-cell patches (16384), 4 ppc, 20 keV, fp64, 6 steps")
    wl = W.uniform_2d(n=(512, 512), patch=(4, 4), ppc=4, T_keV=20.0)
    g = gpu_sim(wl, 64, chunk=24)
    g.step(6)
    o = oracle_run(wl, 6)
    e, b = compare_fields(g, o)
    assert e < 1e-11 and b < 1e-11, (e, b)
    assert np.array_equal(g.counts(), o.counts())
    gx, gu, gw, gid = g.particles()
    ox, ou, ow, oid = o.particles()
    assert np.array_equal(gid, oid)
    for a in range(2):
        assert np.abs(gx[a] - ox[a]).max() < 1e-11
    U, K, pushed = g.history(0, 6)
    assert (pushed == wl["w"].size).all(), pushed
    Uo, Ko = o.energy()
    assert abs(K[5] - Ko) <= 1e-12 * abs(Ko)


def test_maxwell_only_matches_oracle_fp64():
    _announce("vacuum fields 96x64 fp64, 20 steps")
    grid = dict(ndim=2, n=[96, 64], d=[0.1, 0.13], dt=W.cfl_dt((0.1, 0.13)), patch=[16, 16],
                periodic=[1, 1], q=-1.0, m=1.0)
    from paper_1511_03878_amd.sim import Sim
    g = Sim(grid, 64)
    g.set_particles([np.zeros(0), np.zeros(0)], [np.zeros(0)] * 3, np.zeros(0))
    o = oracle.Sim(grid)
    rng = np.random.default_rng(11)
    for c in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        f = rng.standard_normal((64, 96))
        g.set_field(c, f)
        o.set_field(c, f)
    g.step(20)
    o.step(20)
    e, b = compare_fields(g, o)
    assert e < 1e-12 and b < 1e-12, (e, b)


def _rebin_case(grid, wl_kw, seed):
    wl = W.uniform_2d(**wl_kw)
    wl["grid"].update(grid)
    from paper_1511_03878_amd.sim import Sim
    g = Sim(wl["grid"], 64)
    g.set_particles(wl["x"], wl["u"], wl["w"])
    counts = g.counts()
    _, _, _, ids = g.particles()
    rng = np.random.default_rng(seed)
    N = ids.size
    codes = np.full(N, 4, dtype=np.uint8)
    r = rng.random(N)
    moving = r < 0.3
    codes[moving] = rng.integers(0, 9, moving.sum())
    codes[r > 0.97] = 255
    n = wl["grid"]["n"]
    P = wl["grid"]["patch"]
    np_ = (n[0] // P[0], n[1] // P[1])
    owner = np.repeat(np.arange(counts.size), counts)
    dest = np.array([-1 if c == 255 else neighbour_patch(p, int(c), np_, (1, 1))
                     for p, c in zip(owner, codes)], dtype=np.int32)
    newcount, src = oracle.rebin(counts, dest)
    g.rebin_codes(codes)
    assert np.array_equal(g.counts(), newcount)
    _, _, _, gids = g.particles()
    assert np.array_equal(gids, ids[src])


@pytest.mark.parametrize("case", ["4x4_patches", "self_neighbour_1x2", "two_patch_periodic"])
def test_rebin_as_a_function_bit_exact(case):
    _announce(f"re-binning as a function: {case}")
    if case == "4x4_patches":
        _rebin_case(dict(patch=[16, 16]), dict(n=(64, 64), patch=(16, 16), ppc=4), 1)
    elif case == "self_neighbour_1x2":
        _rebin_case(dict(patch=[32, 16]), dict(n=(32, 32), patch=(32, 16), ppc=4), 2)
    else:
        _rebin_case(dict(patch=[16, 32]), dict(n=(32, 32), patch=(16, 32), ppc=4), 3)


def test_lwfa_small_fp64_matches_oracle():
    _announce("lwfa 512x128 fp64, 60 steps (laser through x=0, open x)")
    wl = W.lwfa_2d_small(nsteps=60)
    g = gpu_sim(wl, 64)
    g.step(60)
    o = oracle_run(wl, 60)
    e, b = compare_fields(g, o)
    assert e < 1e-11 and b < 1e-11, (e, b)
    assert np.array_equal(g.counts(), o.counts())
    assert g.diag()["removed"] == o.removed


def test_capacity_growth_keeps_state_exact():
    _announce("capacity growth: tiny slack, 12 steps fp64")
    wl = W.uniform_2d(n=(64, 64), patch=(16, 16), ppc=8, T_keV=200.0)
    g = gpu_sim(wl, 64, capacity_factor=1.0, min_capacity=64)
    g.step(12)
    o = oracle_run(wl, 12)
    e, b = compare_fields(g, o)
    assert e < 1e-11 and b < 1e-11
    assert np.array_equal(g.counts(), o.counts())
    assert np.array_equal(g.particles()[3], o.particles()[3])
    assert g.diag()["relayouts"] >= 1


def test_empty_simulation_steps():
    _announce("empty simulation")
    grid = dict(ndim=2, n=[64, 32], d=[0.1, 0.1], dt=0.05, patch=[16, 16], periodic=[1, 1],
                q=-1.0, m=1.0)
    from paper_1511_03878_amd.sim import Sim
    g = Sim(grid, 32)
    g.set_particles([np.zeros(0), np.zeros(0)], [np.zeros(0)] * 3, np.zeros(0))
    g.step(3)
    assert g.diag()["step"] == 3 and g.num_particles() == 0


@pytest.mark.parametrize("case", ["uniform_fp64", "lwfa_fp32", "blob3d_fp64"])
def test_checkpoint_round_trip_and_resume(case):
    """Save after k steps and restore into a fresh handle: saving again gives
    the same bytes; stepping on matches the uninterrupted run (float atomics
    reorder sums, so FP64 within 1e-12 with exact counts and ids, FP32 within
    1e-5)."""
    _announce(f"checkpoint / resume: {case}")
    if case == "uniform_fp64":
        wl, prec, k, m = W.uniform_2d(n=(64, 64), patch=(16, 16), ppc=4, T_keV=50.0), 64, 7, 6
    elif case == "lwfa_fp32":
        wl, prec, k, m = W.to_float32_state(W.lwfa_2d_small(nsteps=40)), 32, 20, 15
    else:
        wl, prec, k, m = W.blob_3d(n=(32, 16, 16), d=(0.1, 0.1, 0.1), patch=(8, 8, 4), ppc0=2,
                                   blob_radius=4.0, T_keV=30.0), 64, 4, 5
    ref = gpu_sim(wl, prec)
    ref.step(k + m)
    a = gpu_sim(wl, prec)
    a.step(k)
    blob = a.save_state()
    a.close()
    from paper_1511_03878_amd.sim import Sim
    b = Sim(wl["grid"], prec)
    b.load_state(blob)
    assert b.save_state() == blob
    if wl.get("laser"):
        b.add_laser(wl["laser"])
    b.step(m)
    tol = 1e-12 if prec == 64 else 1e-5
    comps = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")
    assert rel_l2([b.field(c) for c in comps], [ref.field(c) for c in comps]) < tol
    assert b.diag()["step"] == ref.diag()["step"] == k + m
    Ub, Kb, _ = b.history(k, m)
    Ur, Kr, _ = ref.history(k, m)
    assert np.allclose(Ub, Ur, rtol=100 * tol, atol=0) and np.allclose(Kb, Kr, rtol=100 * tol, atol=0)
    if prec == 64:
        assert np.array_equal(b.counts(), ref.counts())
        assert np.array_equal(b.particles()[3], ref.particles()[3])
    else:
        assert b.counts().sum() == ref.counts().sum()


def test_graph_replays_match_plain_launches():
    """32-step batches replayed from a captured graph, with host reads and
    synchronisations between replays, equal plain launches after every
    replay (FP64); a capacity-growth run under graphs still matches the
    oracle (tables rebuilt, graph captured again)."""
    _announce("graph replay vs plain launches, fp64")
    wl = W.uniform_2d(n=(64, 64), patch=(16, 16), ppc=4, T_keV=50.0)
    plain = gpu_sim(wl, 64)
    graph = gpu_sim(wl, 64, graph=1)
    for r in range(3):
        plain.step(32)
        graph.step(32)
        assert graph.diag()["step"] == plain.diag()["step"] == 32 * (r + 1)
        comps = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")
        assert rel_l2([graph.field(c) for c in comps], [plain.field(c) for c in comps]) < 1e-12
        assert np.array_equal(graph.counts(), plain.counts())
        assert np.array_equal(graph.particles()[3], plain.particles()[3])
    _announce("graph replay with capacity growth vs oracle, fp64 64 steps")
    wl = W.uniform_2d(n=(64, 64), patch=(16, 16), ppc=8, T_keV=200.0)
    g = gpu_sim(wl, 64, capacity_factor=1.0, min_capacity=64, graph=1)
    g.step(64)
    o = oracle_run(wl, 64)
    e, b = compare_fields(g, o)
    assert e < 1e-11 and b < 1e-11
    assert np.array_equal(g.counts(), o.counts())
    assert np.array_equal(g.particles()[3], o.particles()[3])
    assert g.diag()["relayouts"] >= 1


def test_autotune_restores_state_and_caches(tmp_path):
    _announce("autotune: state restored, settings cached")
    wl = W.lwfa_2d_small(nsteps=200)
    g = gpu_sim(wl, 32)
    g.step(30)
    before = [g.field(c) for c in ("Ex", "Ey", "Bz")] + [g.particles()[3], g.counts()]
    cache = str(tmp_path / "tune.txt")
    r = g.autotune(steps=4, cache=cache)
    assert r["from_cache"] == 0 and r["trials"] >= 8
    assert r["block"] in (256, 512, 1024) and 0 <= r["field_tile"] <= 5 and 1 <= r["lane_stride"] <= 64
    after = [g.field(c) for c in ("Ex", "Ey", "Bz")] + [g.particles()[3], g.counts()]
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    assert g.diag()["step"] == 30
    g.step(10)  # the tuned settings run
    assert g.diag()["step"] == 40
    h = gpu_sim(wl, 32)
    r2 = h.autotune(steps=4, cache=cache)
    assert r2["from_cache"] == 1 and r2["trials"] == 0
    assert (r2["block"], r2["field_tile"], r2["lane_stride"], r2["chunk"]) == \
        (r["block"], r["field_tile"], r["lane_stride"], r["chunk"])


def test_curve_ordered_queue_matches_id_order():
    """Queueing equal-size work items along the Hilbert curve (patch_order = 1,
    section 3.1) only changes which workgroup pushes which patch and when:
    occupancy counts and the particle permutation stay bit-exact and the
    fields agree to rounding (FP64 laser box of 16 x 4 patches, 20 steps)."""
    from paper_1511_03878_amd.sim import Sim
    wl = W.lwfa_2d_small(nsteps=40)
    a = Sim.from_workload(wl, precision=64)
    b = Sim.from_workload(wl, precision=64, patch_order=1)
    a.step(20)
    b.step(20)
    assert np.array_equal(a.counts(), b.counts())
    assert np.array_equal(a.particles()[3], b.particles()[3])
    comps = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")
    assert rel_l2([b.field(c) for c in comps], [a.field(c) for c in comps]) < 1e-12
    a.close()
    b.close()
