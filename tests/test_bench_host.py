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


def test_workload_options():
    wl = {"ppc": 4, "column_density": [0.0, 1.0]}
    opts = bench._options("lwfa_window", wl)
    assert opts["window"][0] == 300 and opts["merge"] == (100, 8, 8)
    assert bench._options("periodic_hi", {})["tune"] == {"maxwell_order": 6}
    assert bench._options("lwfa", {}) == {} and bench._options("blob3d", {}) == {}


def test_headline_is_the_largest_configuration():
    """The default workload is the 3-D box of 512 x 256 x 256 cells (the
    largest single-GPU configuration), loaded from its description."""
    wl, desc = bench._workload("blob3d")
    assert wl["grid"]["n"] == [512, 256, 256] and wl["grid"]["ndim"] == 3
    assert wl["species"]["loading"] == "count" and "x" not in wl
    assert desc.startswith("blob_3d: 512x256x256")


def test_traffic_is_reported_only_for_the_measured_source():
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path) as f:
        recs = json.load(f)
    for key, rec in recs.items():
        kernel, workload, prec = key.split("/")
        nd = 3 if kernel == "k_particles3d" else 2
        got = bench._measured_traffic(kernel, workload, int(prec[1:]), nd)
        if rec["source_sha"] == bench._kernel_source_sha(nd):
            assert got == rec["traffic_bytes_per_launch"]
        else:
            assert got is None
    assert bench._measured_traffic("k_particles2d", "no_such_workload", 32, 2) is None


def test_smoke_workload_loads_in_the_oracle():
    """__graft_entry__.smoke() loads its thermal box from the species
    description on both sides; the oracle's loader must accept it (host)."""
    import oracle
    from paper_1511_03878_amd import workloads as W
    wl = W.uniform_2d(n=(64, 64), patch=(16, 16), ppc=8)
    o = oracle.Sim(wl["grid"])
    o.particles_init(wl["species"])
    assert o.particles()[2].size == 64 * 64 * 8
