"""Host logic of bench.py (no GPU): the one-GPU guard, the per-workload
options, the algorithmic bytes per particle-step and the traffic lookup."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


@pytest.mark.parametrize("nd,prec", [(2, 32), (2, 64), (3, 32), (3, 64)])
def test_bytes_per_particle_step_from_the_particle_layout(nd, prec):
    # read nd positions, 3 momenta and the weight; write nd positions and 3 momenta
    t = prec // 8
    assert bench.BYTES_PER_PARTICLE_STEP[(nd, prec)] == t * ((nd + 3 + 1) + (nd + 3))


class _Rec:
    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        return lambda *a: self.calls.append((name, a))


def test_workload_options_reach_both_sides():
    wl = {"ppc": 4, "column_density": [0.0, 1.0]}
    g, o = _Rec(), _Rec()
    opts = bench._options("lwfa_window", wl)
    bench._apply(g, opts)
    bench._apply(o, opts, oracle_side=True)
    assert [c[0] for c in g.calls] == ["set_window", "set_merge"] == [c[0] for c in o.calls]
    hi = bench._options("periodic_hi", {})
    assert hi["tune"] == {"maxwell_order": 6}
    o = _Rec()
    bench._apply(o, hi, oracle_side=True)
    assert o.calls == [("set_maxwell_order", (6,))]
    assert bench._options("lwfa", {}) == {}


def test_traffic_is_reported_only_for_the_measured_source():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)["k_particles2d/lwfa/f32"]
    got = bench._measured_traffic(32, "lwfa")
    if rec["source_sha"] == bench._kernel_source_sha():
        assert got == rec["traffic_bytes_per_launch"]
    else:
        assert got is None
    assert bench._measured_traffic(32, "no_such_workload") is None
