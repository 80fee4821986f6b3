"""Batched multi-simulation stepping and the serving loop on the GPU.

A simulation stepped inside a batch (one queue, one launch per kernel for all
members) must give the same result as the same simulation stepped alone:
FP64 within 1e-12 relative L2 on the fields with bit-exact patch occupancy
and particle order (only the order of floating-point atomic additions can
differ), FP32 within 1e-5 after a few steps.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_1511_03878_amd import serve
from tests import fixtures as W
from paper_1511_03878_amd.sim import Batch, Sim
from tests.helpers import B_COMPS, E_COMPS, rel_l2

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _members():
    # uneven sizes, different patch sizes, periodic and open boundaries
    return [
        (W.lwfa_2d_small(nsteps=40, n=(256, 64), patch=(32, 32)), 40),
        (W.uniform_2d(n=(64, 64), patch=(16, 16), ppc=4, T_keV=20.0), 25),
        (W.lwfa_2d_small(nsteps=40, n=(512, 128), patch=(32, 32)), 33),
        (W.uniform_2d(n=(96, 32), patch=(16, 16), ppc=2, T_keV=50.0), 40),
    ]


def _fields(s):
    return [s.field(c) for c in E_COMPS + B_COMPS]


@pytest.mark.parametrize("precision", [64, 32])
def test_batch_matches_alone(precision):
    _announce(f"batch of 4 uneven simulations vs alone, fp{precision}")
    members = _members()
    if precision == 32:
        members = [(W.to_float32_state(wl), min(n, 3)) for wl, n in members]
    alone = []
    for wl, n in members:
        s = Sim.from_workload(wl, precision=precision)
        s.step(n)
        alone.append((_fields(s), s.counts(), s.particles()[3], s.diag()))
        s.close()
    b = Batch(precision)
    sims = []
    for wl, n in members:
        s = Sim.from_workload(wl, precision=precision)
        b.add(s, n)
        sims.append(s)
    done = 0
    for _ in range(20):
        done += b.step(8)
        if done == len(sims):
            break
    assert done == len(sims)
    assert sorted(x.handle.value for x in b.finished()) == sorted(x.handle.value for x in sims)
    tol = 1e-12 if precision == 64 else 1e-5
    for (wl, n), s, (fa, ca, ia, da) in zip(members, sims, alone):
        d = s.diag()
        assert d["step"] == n == da["step"]
        assert rel_l2(_fields(s), fa) < tol
        assert np.array_equal(s.counts(), ca)
        if precision == 64:
            assert np.array_equal(s.particles()[3], ia)


def test_batch_members_can_join_and_leave_between_slices():
    _announce("continuous batching: join/leave between slices (fp64)")
    members = _members()
    b = Batch(64)
    first = Sim.from_workload(members[0][0], precision=64)
    b.add(first, 40)
    b.step(10)
    late = Sim.from_workload(members[1][0], precision=64)
    b.add(late, 25)
    for _ in range(10):
        b.step(10)
        for s in b.finished():
            b.remove(s)
        if len(b) == 0:
            break
    assert len(b) == 0
    ref0 = Sim.from_workload(members[0][0], precision=64)
    ref0.step(40)
    ref1 = Sim.from_workload(members[1][0], precision=64)
    ref1.step(25)
    assert rel_l2(_fields(first), _fields(ref0)) < 1e-12
    assert rel_l2(_fields(late), _fields(ref1)) < 1e-12
    assert first.diag()["step"] == 40 and late.diag()["step"] == 25


def test_serving_admits_under_budget_and_results_match_alone():
    _announce("serving: 6 requests, small budget forces queueing (fp32)")
    reqs = serve.make_requests(6, rate=50.0, steps_range=(20, 60), scan_patch=32)
    for r in reqs:  # keep the test small: shrink the grids
        r.params = dict(r.params, n=(min(r.params["n"][0], 512), min(r.params["n"][1], 128)))
    sizes = []
    for r in reqs:
        wl = serve.make_workload(r)
        from paper_1511_03878_amd.sim import estimate_bytes
        sizes.append(estimate_bytes(wl["grid"], 32, serve.particle_count(wl)))
    budget = int(max(sizes) * 1.6)  # at most one or two residents at a time
    srv = serve.Server(budget, precision=32, slice_steps=10)
    report = srv.run(reqs, realtime=False)
    assert report["requests"] == 6
    assert all(r.done is not None and r.done >= r.arrival for r in reqs)
    assert srv.in_use == 0 and len(srv.batch) == 0
    # queueing happened: some request was admitted after it arrived
    assert any(r.admitted > r.arrival for r in reqs)
    # each result equals the same request run alone (FP32: atomics reorder sums)
    for r in reqs[:3]:
        wl = serve.make_workload(r)
        s = Sim.from_workload(wl, precision=32)
        s.step(r.nsteps)
        assert s.diag()["step"] == r.result["diag"]["step"] == r.nsteps
        assert rel_l2([s.field("Ey"), s.field("Bz")], [r.result["Ey"], r.result["Bz"]]) < 1e-4
        U, K, _ = s.history(0, r.nsteps)
        assert np.allclose(U, r.result["U"], rtol=1e-4, atol=1e-9 * max(1.0, abs(U).max()))


def test_served_results_match_the_oracle_and_growth_is_charged():
    """Requests served together (continuous batching, FP32, loaded on the
    device from their descriptions) against the oracle run from the same
    descriptions rounded to FP32 storage: one-step requests' fields within
    1e-5, 120-step requests' energy histories within 1e-3.  Patches are
    sized without slack, so capacities grow while the requests are resident,
    and the server charges each resident what it really holds."""
    _announce("served vs oracle: 4 requests fp32, capacity growth charged")
    from tests.helpers import oracle_sim
    reqs = serve.make_requests(4, rate=100.0, steps_range=(1, 1), scan_patch=32)
    for k, r in enumerate(reqs):
        r.params = dict(r.params, n=(min(r.params["n"][0], 320), min(r.params["n"][1], 128)), a0=6.0)
        r.nsteps = 1 if k % 2 == 0 else 120
    tune = {"capacity_factor": 1.0, "min_capacity": 64}

    def result(sim):
        d = sim.diag()
        U, K, _ = sim.history(0, d["step"])
        return {"diag": d, "U": U, "K": K, "held": sim.device_bytes(),
                "fields": [sim.field(c) for c in ("Ex", "Ey", "Bz")]}

    srv = serve.Server(int(64 * 2**30), precision=32, slice_steps=5, result_fn=result, tune=tune)
    srv.run(reqs, realtime=False)
    assert srv.in_use == 0
    # every charge covered what the residents held, estimate or more
    assert all(charged >= held for _, charged, held in srv.charges)
    assert max(n for n, _, _ in srv.charges) >= 2  # requests shared the GPU
    # capacities grew while requests were resident (the server saw it)
    grew = [r for r in reqs if r.result["diag"]["relayouts"] > 0]
    assert grew and srv.peak_in_use >= max(r.result["held"] for r in grew)
    for r in reqs:
        wl = serve.make_workload(r)
        o = oracle_sim(wl, storage=32)
        Wo = []
        for _ in range(r.nsteps):
            o.step(1)
            Wo.append(sum(o.energy()))
        if r.nsteps == 1:
            ref = [o.field(c)[0] for c in ("Ex", "Ey", "Bz")]
            assert rel_l2(r.result["fields"], ref) < 1e-5
        Wg = r.result["U"] + r.result["K"]
        assert np.abs(Wg - np.array(Wo)).max() <= 1e-3 * max(np.abs(Wo).max(), 1e-300)
