"""Benchmark: particle-steps/s of the patch-PIC step on one MI355X.

A step is one pass of the whole hot path over the resident state: work-queue
build, fused gather / Boris / move / Esirkepov deposit, Yee update with its
face conditions, and the per-patch re-binning.  All inputs are seeded and
synthetic and are loaded on the device from their descriptions.

The headline workload is the largest single-GPU configuration, the 3-D box
(512 x 256 x 256 cells, density n0 (1 + 0.9 cos kx) plus a 4 n0 sphere of
radius 20 cells, round(8 n / n0) electrons per cell, 10 keV, periodic, FP32;
2.7e8 particles).  The timed region covers exactly --steps steps of the
instance that ran the --warmup steps (inputs already in HBM), bracketed by
device synchronisations.

Further measurements on the same JSON line (each on its own instance, after
the headline):
  lwfa_late     -- the 4096 x 1024 laser-wakefield box (FP32), timed over the
                   steps after step 1000, once the pulse has formed a wake
                   and patch occupancy is uneven;
  batched_scan  -- 64 laser-wakefield simulations of uneven size, 500 steps
                   each, stepped in one batch against the same simulations
                   run one at a time;
  served_scan   -- Poisson arrivals (4/s) of such simulations with 200..2000
                   steps each, admitted against a 200 GiB HBM budget and
                   stepped with continuous batching: 20 warm-up requests, then
                   400 measured (p50 / p99 time-to-result), plus the same
                   requests served in compressed time with continuous batching
                   and one at a time;
  cpu_baseline  -- the FP64 oracle (OpenMP timing build) on a sample of the
                   headline workload on this host, at 1 thread and all threads.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec (gather+push+deposit+Maxwell) & % HBM peak; batched p50/p99"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per particle-step of the fused particle kernel: read the
# position (2 or 3 components), momentum (3) and weight, write position and
# momentum
BYTES_PER_PARTICLE_STEP = {(2, 32): 44, (2, 64): 88, (3, 32): 52, (3, 64): 104}
S6 = 75 / 64 + 25 / 384 + 3 / 640   # the sixth-order solver's stability factor


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# workloads

def _workload(name):
    from paper_1511_03878_amd import workloads as W
    if name == "blob3d":
        wl = W.blob_3d(patch=(8, 8, 8))
        desc = ("blob_3d: 512x256x256 cells (dx=0.1 c/w_p), periodic, n = n0 (1 + 0.9 cos kx) plus a "
                "4 n0 sphere of radius 20 cells, round(8 n/n0) electrons per cell (2.7e8), 10 keV, "
                "FP32; each 16^3-cell patch of the configuration run as eight 8^3 GPU patches")
    elif name == "lwfa":
        wl = W.lwfa_2d()
        desc = ("lwfa_2d: 4096x1024 cells (dx=lambda/32, dy=lambda/8), 32x32-cell patches, 4 ppc "
                "electrons behind a 2->12 lambda ramp to 0.003 n_c (16.5M), a0=4 w0=12 lambda "
                "Gaussian laser through x=0, open x / periodic y")
    elif name == "lwfa_window":
        wl = W.lwfa_2d()
        desc = ("lwfa_2d with a moving window from step 300 and particle merging every 100 steps "
                "(cells above 8 particles, 8 k-means rounds)")
    elif name == "periodic_hi":
        wl = W.uniform_2d(n=(4096, 1024), patch=(32, 32), ppc=4, T_keV=1.0, cfl=0.9 / S6)
        desc = "uniform_2d 4096x1024, 4 ppc, 1 keV, sixth-order field solver"
    elif name == "uniform":
        wl = W.uniform_2d()
        desc = "uniform_2d: 128x128 cells, 16x16-cell patches, 16 ppc, 1 keV, periodic"
    else:
        raise SystemExit(f"unknown workload {name}")
    return wl, desc


def _options(name, wl):
    if name == "lwfa_window":
        return {"window": (300, 1.0, (wl["ppc"], 1), wl["column_density"]), "merge": (100, 8, 8)}
    if name == "periodic_hi":
        return {"tune": {"maxwell_order": 6}}
    return {}


def _sim_for(wl, name, precision, **extra):
    from paper_1511_03878_amd.sim import Sim
    opts = _options(name, wl)
    sim = Sim.from_workload(wl, precision=precision, **opts.get("tune", {}), **extra)
    if "window" in opts:
        sim.set_window(*opts["window"])
    if "merge" in opts:
        sim.set_merge(*opts["merge"])
    return sim


# ---------------------------------------------------------------------------
# roofline pieces

def _kernel_source_sha(ndim):
    h = hashlib.sha256()
    files = ("k_particles3d.hip",) if ndim == 3 else ("k_particles.hip",)
    for f in files + ("particle_common.h", "pic_dev.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1511_03878_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _measured_traffic(kernel, workload, precision, ndim):
    """HBM bytes per launch of the particle kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE measurement, if it was taken on the current
    kernel source in the same window (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(f"{kernel}/{workload}/f{precision}")
    if not rec or rec.get("source_sha") != _kernel_source_sha(ndim):
        return None
    return rec.get("traffic_bytes_per_launch")


def _roofline(timing, total, ndim, precision, workload, breakdown):
    ms, launches = timing["particles"]
    avg_s = ms / 1e3 / max(launches, 1)
    per_launch = BYTES_PER_PARTICLE_STEP[(ndim, precision)] * total / max(launches, 1)
    achieved = per_launch / avg_s / 1e9
    kernel = "k_particles2d" if ndim == 2 else "k_particles3d"
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": _measured_traffic(kernel, workload, precision, ndim),
            "kernel": kernel, "algorithmic_bytes_per_launch": per_launch,
            "kernel_ms_per_launch": round(avg_s * 1e3, 4), "launches": launches,
            "kernel_ms_per_launch_after_timed_region": breakdown}


def _timed_window(sim, steps, ndim, precision, workload, kernel_timing=True):
    """Time `steps` steps of `sim` (particle kernel timed by its own dispatch
    events); returns (particle-steps/s, ms/step, pushed, roofline)."""
    import torch
    step0 = sim.diag()["step"]
    if kernel_timing:
        sim.timing_enable("particles")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    _, _, pushed = sim.history(step0, steps)
    total = int(pushed.sum())
    roof = None
    if kernel_timing:
        timing = sim.timing()
        sim.timing_enable(True)
        sim.step(min(16, max(1, steps // 4)))
        breakdown = {k: round(v[0] / max(v[1], 1), 4) for k, v in sim.timing().items()}
        sim.timing_enable(False)
        roof = _roofline(timing, total, ndim, precision, workload, breakdown)
    return total / wall, wall * 1e3 / steps, total, roof


def _imbalance(sim):
    """The paper's imbalance measure (section 3.1, Fig. 4) on one more step
    with per-item stamps: max / mean busy time of the compute units with the
    work queue, and with the same item times dealt out as fixed domains."""
    sim.timing_enable("stamps")
    sim.step(1)
    r = sim.imbalance()
    sim.timing_enable(False)
    keep = ("imbalance", "static_imbalance", "segment_imbalance", "units", "items", "span_us",
            "busy_max_us", "busy_mean_us", "patch_max_us", "patch_mean_us")
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items() if k in keep}


# ---------------------------------------------------------------------------
# extra measurements

def _det_window(wl, args):
    """The headline workload again with deterministic deposition (same warm-up
    and window): the cost of bitwise-reproducible currents."""
    import torch
    sim = _sim_for(wl, args.workload, args.precision, deterministic=1)
    if args.pre_steps > 0:
        sim.step(args.pre_steps)
    if args.warmup > 0:
        sim.step(args.warmup)
    sim.sync()
    val, ms, _, roof = _timed_window(sim, args.steps, wl["grid"]["ndim"], args.precision, args.workload,
                                     kernel_timing=not args.no_kernel_timing)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"value": val, "ms_per_step": ms, "unit": "particle-steps/s",
            "kernel_ms_per_launch": roof["kernel_ms_per_launch"] if roof else None,
            "note": "64-bit fixed-point current summed with integer atomics; runs repeat bit for bit"}

def _lwfa_late(precision, pre_steps=1000, steps=200):
    """The laser box timed after its first `pre_steps` steps (wake formed,
    uneven patch occupancy)."""
    wl, desc = _workload("lwfa")
    sim = _sim_for(wl, "lwfa", precision)
    sim.step(pre_steps)
    sim.sync()
    d0 = sim.diag()
    val, ms, total, roof = _timed_window(sim, steps, 2, precision, "lwfa_late")
    d = sim.diag()
    out = {"workload": desc, "steps_before": pre_steps, "steps_timed": steps, "value": val,
           "unit": "particle-steps/s", "ms_per_step": ms, "particles": d["particles"],
           "occupancy": {"min": d0["occupancy_min"], "mean": round(d0["occupancy_mean"], 1),
                         "max": d0["occupancy_max"]},
           "relayouts": d["relayouts"], "roofline": roof, "imbalance": _imbalance(sim)}
    sim.close()
    return out


TUNE_CACHE = os.path.join(ROOT, "_build", "patch_tune.txt")


def _tuned_scan_patch(params, precision):
    """Patch edge and particle-kernel workgroup size of the scan, picked by the
    library's patch tuner on the median-sized draw (the choice applies to
    every member, so one batch shares one kernel specialisation)."""
    from paper_1511_03878_amd import workloads as W
    from paper_1511_03878_amd.sim import autotune_patch
    sizes = [p["n"][0] * p["n"][1] * p["ppc"] for p in params]
    rep = params[sorted(range(len(params)), key=lambda k: sizes[k])[len(params) // 2]]
    os.makedirs(os.path.dirname(TUNE_CACHE), exist_ok=True)
    grid, tune, res = autotune_patch(W.scan_sim(rep), precision, candidates=(16, 32), warm=20, steps=20,
                                     cache=TUNE_CACHE)
    patch = tuple(grid["patch"][:2])
    return patch, tune, {"patch": list(patch), "block": tune["block"], "trials": res["trials"],
                         "from_cache": res["from_cache"], "ms_per_step": res["ms_per_step"],
                         "tuned_on": list(rep["n"])}


def _scan_bench(count, steps, precision):
    """Batched parameter scan: `count` laser-wakefield simulations of uneven
    size stepped together in one batch (one work queue, one persistent
    particle launch per step) against the same simulations run one at a
    time.  Returns aggregate particle-steps/s of both."""
    import torch
    from paper_1511_03878_amd import workloads as W
    from paper_1511_03878_amd.sim import Batch, Sim
    params = W.scan_params(count)
    patch, tune, tuned = _tuned_scan_patch(params, precision)
    wls = [W.scan_sim(p, seed=W.DEFAULT_SEED + k, patch=patch) for k, p in enumerate(params)]
    t_alone, total = 0.0, 0
    for wl in wls:
        s = Sim.from_workload(wl, precision=precision, **tune)
        total += s.num_particles() * steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        t_alone += time.perf_counter() - t0
        s.close()
    sims = [Sim.from_workload(wl, precision=precision, **tune) for wl in wls]
    b = Batch(precision)
    for s in sims:
        b.add(s, steps)
    b.step(0)  # builds the batch tables outside the timed region
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < count:
        done += b.step(steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    for s in sims:
        s.close()
    b.close()
    return {"sims": count, "steps_each": steps, "particle_steps": total,
            "batched": total / t_batch, "one_at_a_time": total / t_alone,
            "speedup": t_alone / t_batch, "unit": "particle-steps/s", "launch": "one batch, one "
            "persistent particle launch per step over every member's patches", "autotuned": tuned,
            "grids": [list(p["n"]) for p in params][:8] + (["..."] if count > 8 else [])}


def _serve_bench(count, warm, rate, steps_range, budget_gb, precision, compare, compare_rate):
    """Served scan: Poisson arrivals admitted against an HBM budget and
    stepped with continuous batching (real time; the first `warm` requests
    are warm-up); then `compare` requests arriving at `compare_rate` per
    second (faster than one request at a time can be served, so that the
    comparison measures service capacity rather than the arrival rate), in
    compressed time (idle gaps skipped), with continuous batching and one at
    a time."""
    from paper_1511_03878_amd import serve
    from paper_1511_03878_amd import workloads as W
    reqs = serve.make_requests(count + warm, rate, steps_range=steps_range)
    patch, tune, tuned = _tuned_scan_patch(W.scan_params(64), precision)
    budget = int(budget_gb * 2**30)
    srv = serve.Server(budget, precision=precision, slice_steps=25, result_fn=lambda sim: {},
                       patch=patch, tune=tune)
    rep = srv.run(reqs, realtime=True, warmup=warm)
    rep.update({"rate_per_s": rate, "steps_range": list(steps_range), "budget_GiB": budget_gb,
                "warmup_requests": warm, "unit": "particle-steps/s", "autotuned": tuned})
    if compare > 0:
        cmp = {}
        for label, members in (("continuous_batching", 256), ("one_at_a_time", 1)):
            rq = serve.make_requests(compare, compare_rate, steps_range=steps_range)
            s2 = serve.Server(budget, precision=precision, slice_steps=25, result_fn=lambda sim: {},
                              max_members=members, patch=patch, tune=tune)
            r = s2.run(rq, realtime=False)
            cmp[label] = {"throughput": r["throughput"], "ttr_p50_s": r["ttr_p50_s"],
                          "ttr_p99_s": r["ttr_p99_s"], "wall_s": r["wall_s"]}
        cmp["speedup"] = cmp["continuous_batching"]["throughput"] / cmp["one_at_a_time"]["throughput"]
        cmp["requests"] = compare
        cmp["rate_per_s"] = compare_rate
        cmp["note"] = "compressed time: idle gaps before an arrival are skipped"
        rep["compressed_comparison"] = cmp
    return rep


def _cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def _cpu_baseline(budget_s=25.0):
    """The FP64 oracle (timing build: -O3 -march=native, OpenMP particle loop
    with per-thread current arrays) on a 128 x 64 x 64 box with the headline's
    density profile and cell size, at 1 thread and at every host thread."""
    import oracle
    from paper_1511_03878_amd import workloads as W
    oracle.use_timing_build()
    wl = W.blob_3d(n=(128, 64, 64), patch=(8, 8, 8), blob_radius=20.0)
    res = {}
    nproc = os.cpu_count() or 1
    for th in (1, nproc):
        got = oracle.set_threads(th)
        o = oracle.Sim(wl["grid"])
        o.particles_init(wl["species"])
        n = o.particles()[2].size
        steps, t0 = 0, time.perf_counter()
        while True:
            o.step(1)
            steps += 1
            if time.perf_counter() - t0 > budget_s / 4 or steps >= 3:
                break
        dt = time.perf_counter() - t0
        res[th] = (n * steps / dt, got, steps, n, dt)
        del o
    best = res[nproc]
    return {"value": best[0], "unit": "particle-steps/s", "cores": best[1], "kind": "oracle",
            "cpu_model": _cpu_model(), "value_1_thread": res[1][0],
            "sample": (f"{best[2]} step(s) of a 128x64x64 box with the headline's profile "
                       f"({best[3]} particles), FP64 oracle timing build (-O3 -march=native, OpenMP), "
                       f"{best[4]:.1f} s at {best[1]} threads; {res[1][2]} step(s) at 1 thread "
                       f"{res[1][4]:.1f} s")}


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--workload", default="blob3d")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-late", action="store_true")
    ap.add_argument("--scan", type=int, default=64, metavar="N",
                    help="batched scan of N simulations vs one at a time (0: skip)")
    ap.add_argument("--scan-steps", type=int, default=500)
    ap.add_argument("--serve", type=int, default=400, metavar="N",
                    help="serve N Poisson-arriving requests after the warm-up ones (0: skip)")
    ap.add_argument("--serve-warmup", type=int, default=20)
    ap.add_argument("--serve-compare", type=int, default=100)
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-compare-rate", type=float, default=40.0)
    ap.add_argument("--serve-steps", default="200,2000")
    ap.add_argument("--pre-steps", type=int, default=0,
                    help="untimed steps of the headline instance before its warm-up (e.g. the laser "
                         "box after step 1000)")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--deterministic", action="store_true",
                    help="run the headline with deterministic deposition (fixed-point current "
                         "accumulators, bitwise reproducible)")
    ap.add_argument("--no-det", action="store_true",
                    help="skip the extra window of the headline workload in deterministic mode")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first time an elementwise kernel that reads and writes MIB MiB (calibrates "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE against a known byte count)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    copy_cal = None
    if args.copy_calibration > 0:
        # an elementwise kernel that reads MIB MiB and writes MIB MiB (a
        # same-dtype copy_ would go to the DMA engines, not to a kernel)
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.full((n,), 1.0, device="cuda", dtype=torch.float32)
        b = torch.empty_like(a)
        torch.mul(a, 1.5, out=b)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.mul(a, 1.5, out=b)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        copy_cal = {"kernel": "elementwise mul", "bytes_read": 4 * n, "bytes_written": 4 * n, "ms": ms,
                    "GBps": 8 * n / ms / 1e6}
        del a, b
    wl, desc = _workload(args.workload)
    ndim = wl["grid"]["ndim"]
    t_setup = time.perf_counter()
    sim = _sim_for(wl, args.workload, args.precision, deterministic=int(args.deterministic))
    sim.sync()
    _log(f"workload loaded on the device in {time.perf_counter() - t_setup:.1f} s: {desc}")
    if args.pre_steps > 0:
        sim.step(args.pre_steps)
        sim.sync()
    if args.warmup > 0:
        sim.step(args.warmup)
        sim.sync()
    _log(f"timing {args.steps} steps")
    value, ms_step, total, roof = _timed_window(sim, args.steps, ndim, args.precision, args.workload,
                                                kernel_timing=not args.no_kernel_timing)
    d = sim.diag()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "steps_timed": args.steps, "particles": int(d["particles"]),
                   "occupancy": {"min": d["occupancy_min"], "mean": round(d["occupancy_mean"], 1),
                                 "max": d["occupancy_max"]},
                   "relayouts": d["relayouts"]},
        "roofline": roof,
        "imbalance": _imbalance(sim),
    }
    if args.pre_steps:
        out["config"]["steps_before_warmup"] = args.pre_steps
    out["config"]["deterministic"] = bool(args.deterministic)
    if copy_cal:
        out["copy_calibration"] = copy_cal
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if not args.no_det and not args.deterministic:
        _log("headline workload in deterministic mode")
        out["deterministic_mode"] = _det_window(wl, args)
    if not args.no_late:
        _log("laser box after step 1000")
        out["lwfa_late"] = _lwfa_late(args.precision)
    if args.scan > 0:
        _log(f"batched scan of {args.scan} simulations x {args.scan_steps} steps")
        out["batched_scan"] = _scan_bench(args.scan, args.scan_steps, args.precision)
    if args.serve > 0:
        lo, hi = (int(v) for v in args.serve_steps.split(","))
        _log(f"serving {args.serve_warmup} + {args.serve} requests")
        out["served_scan"] = _serve_bench(args.serve, args.serve_warmup, args.serve_rate, (lo, hi),
                                          200.0, args.precision, args.serve_compare,
                                          args.serve_compare_rate)
    if not args.no_cpu:
        _log("timing the CPU oracle")
        out["cpu_baseline"] = _cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
