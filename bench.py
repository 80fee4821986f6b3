"""Benchmark: particle-steps/s of the full 2-D patch-PIC step on one MI355X.

A step is one pass of the whole hot path over the resident state: work-queue
build, fused gather / Boris / move / Esirkepov deposit, fused Yee update with
the laser-driven and outflow faces, and the per-patch re-binning.  The
workload is the laser-wakefield box (4096 x 1024 cells, 32 x 32-cell patches,
4 electrons per plasma cell behind a linear density ramp, a0 = 4 Gaussian
laser driven through x = 0), all inputs seeded and synthetic.

Prints one JSON line.  The timed region covers exactly --steps steps of a
freshly loaded simulation (inputs already in HBM), bracketed by device
synchronisations; --warmup steps run first on a separate instance.
"""
from __future__ import annotations

import argparse
import json
import math
import os
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


# per-workload options applied to the simulation (and to the oracle for the
# CPU baseline): descriptor settings, moving window, merging
S6 = 75 / 64 + 25 / 384 + 3 / 640   # the sixth-order solver's stability factor


def _options(name, wl):
    if name == "lwfa_window":
        return {"window": (300, 1.0, (wl["ppc"], 1), wl["column_density"]), "merge": (100, 8, 8)}
    if name == "periodic_hi":
        return {"tune": {"maxwell_order": 6}}
    return {}


def _apply(sim, opts, oracle_side=False):
    if "window" in opts:
        sim.set_window(*opts["window"])
    if "merge" in opts:
        sim.set_merge(*opts["merge"])
    if oracle_side and opts.get("tune", {}).get("maxwell_order") == 6:
        sim.set_maxwell_order(6)


def _workload(name, steps):
    from paper_1511_03878_amd import workloads as W
    if name == "lwfa_window":
        wl = W.lwfa_2d(nsteps=max(steps, 1))
        desc = ("lwfa_2d with a moving window from step 300 (v = c, jumps of one 32-cell patch column, "
                "4 ppc cold plasma of the profile injected) and particle merging every 100 steps "
                "(cells above 8 particles, 8 k-means rounds): 4096x1024 cells, 16.5M particles")
    elif name == "periodic_hi":
        wl = W.uniform_2d(n=(4096, 1024), patch=(32, 32), ppc=4, T_keV=1.0, cfl=0.9 / S6)
        desc = ("uniform_2d with the sixth-order field solver: 4096x1024 cells (dx=0.1 c/w_p), "
                "32x32-cell patches, 4 ppc, 1 keV, periodic (16.8M particles)")
    elif name == "lwfa":
        wl = W.lwfa_2d(nsteps=max(steps, 1))
        desc = ("lwfa_2d: 4096x1024 cells (dx=lambda/32, dy=lambda/8), 32x32-cell patches, "
                "4 ppc electrons behind a 2->12 lambda ramp to 0.003 n_c (16.5M particles), "
                "a0=4 w0=12 lambda Gaussian laser through x=0, open x / periodic y")
    elif name == "lwfa_small":
        wl = W.lwfa_2d_small(nsteps=max(steps, 1))
        desc = "lwfa_2d_small: 512x128 cells, 32x32-cell patches, 4 ppc"
    elif name == "blob3d":
        wl = W.blob_3d(patch=(8, 8, 8))
        desc = ("blob_3d: 512x256x256 cells (dx=0.1 c/w_p), periodic, 8x8x8-cell patches "
                "(each 16^3 patch of the configuration as 8 GPU patches), ppc=round(8 n/n0) with "
                f"n = n0 (1 + 0.9 cos kx) and a 4 n0 sphere of radius 20 cells, 10 keV "
                f"({wl['w'].size / 1e6:.1f}M particles)")
    elif name == "uniform":
        wl = W.uniform_2d()
        desc = "uniform_2d: 128x128 cells, 16x16-cell patches, 16 ppc, 1 keV, periodic"
    else:
        raise SystemExit(f"unknown workload {name}")
    return wl, desc


def _sim_for(wl, name, precision):
    from paper_1511_03878_amd.sim import Sim
    opts = _options(name, wl)
    sim = Sim.from_workload(wl, precision=precision, **opts.get("tune", {}))
    _apply(sim, opts)
    return sim


def _kernel_source_sha():
    """Hash of the sources the particle kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("k_particles.hip", "particle_common.h", "pic_dev.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1511_03878_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _measured_traffic(precision, workload):
    """HBM bytes per launch of the particle kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE measurement, if it was taken on the current
    kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(f"k_particles2d/{workload}/f{precision}")
    if not rec or rec.get("source_sha") != _kernel_source_sha():
        return None
    return rec.get("traffic_bytes_per_launch")


def _cpu_baseline(name, budget_s=25.0):
    """Time the FP64 oracle (single-threaded C, as it stands) on one step of
    the same workload on this host."""
    import oracle
    if name == "blob3d":
        # one eighth of the box (256 x 128 x 128 cells, same density profile)
        from paper_1511_03878_amd import workloads as W
        wl = W.blob_3d(n=(256, 128, 128), patch=(8, 8, 8))
    else:
        wl, _ = _workload(name, 1)
    if not os.path.exists(os.path.join(ROOT, "oracle", "liborc.so")):
        oracle.build(force=False)
    o = oracle.Sim(wl["grid"])
    o.set_particles(wl["x"], wl["u"], wl["w"])
    if wl.get("laser"):
        o.set_laser(ey=wl["laser"]["ey"], ez=wl["laser"].get("ez"))
    _apply(o, _options(name, wl), oracle_side=True)
    n = wl["w"].size
    t0 = time.perf_counter()
    steps = 0
    while True:
        o.step(1)
        steps += 1
        if time.perf_counter() - t0 > budget_s / 2 or steps >= 3:
            break
    dt = time.perf_counter() - t0
    return {"value": n * steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} step(s) of {'one eighth of ' if name == 'blob3d' else ''}"
                      f"the workload ({n} particles), FP64 oracle, "
                      f"{dt:.1f} s on one host core"}


def _scan_bench(count, steps, precision, seed=None):
    """Batched parameter scan: `count` laser-wakefield simulations of uneven
    size stepped together in one batch, against the same simulations run one
    at a time.  Returns aggregate particle-steps/s of both."""
    import torch
    from paper_1511_03878_amd import workloads as W
    from paper_1511_03878_amd.sim import Batch, Sim
    params = W.scan_params(count)
    wls = [W.scan_sim(p, steps, seed=W.DEFAULT_SEED + k) for k, p in enumerate(params)]
    total = sum(int(w["w"].size) for w in wls) * steps
    # one at a time
    t_alone = 0.0
    for wl in wls:
        s = Sim.from_workload(wl, precision=precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        t_alone += time.perf_counter() - t0
        s.close()
    # batched
    sims = [Sim.from_workload(wl, precision=precision) for wl in wls]
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
    return {"sims": count, "steps_each": steps, "particle_steps": total,
            "batched": total / t_batch, "one_at_a_time": total / t_alone,
            "speedup": t_alone / t_batch, "unit": "particle-steps/s",
            "grids": [list(p["n"]) for p in params][:8] + (["..."] if count > 8 else [])}


def _serve_bench(count, rate, steps_range, budget_gb, precision):
    """Served scan: Poisson arrivals admitted against an HBM budget and
    stepped with continuous batching; time-to-result percentiles."""
    from paper_1511_03878_amd import serve
    reqs = serve.make_requests(count, rate, steps_range=steps_range)
    srv = serve.Server(int(budget_gb * 2**30), precision=precision, slice_steps=25,
                       result_fn=lambda sim: {"diag": sim.diag()})
    rep = srv.run(reqs, realtime=True)
    rep.update({"rate_per_s": rate, "steps_range": list(steps_range), "budget_GiB": budget_gb,
                "unit": "particle-steps/s"})
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--workload", default="lwfa")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--scan", type=int, default=16, metavar="N",
                    help="also run a batched scan of N simulations vs one at a time (0: skip)")
    ap.add_argument("--scan-steps", type=int, default=100)
    ap.add_argument("--serve", type=int, default=24, metavar="N",
                    help="also serve N Poisson-arriving requests and report p50/p99 (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-steps", default="200,2000")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the run, time a plain device copy of MIB MiB (calibrates "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE against a known byte count)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1511_03878_amd.sim import Sim

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
    wl, desc = _workload(args.workload, args.steps)
    print(f"[bench] workload ready: {desc}", file=sys.stderr, flush=True)

    if args.warmup > 0 and wl["grid"]["ndim"] == 2:
        w = _sim_for(wl, args.workload, args.precision)
        w.step(args.warmup)
        w.sync()
        w.close()
        del w
    sim = _sim_for(wl, args.workload, args.precision)
    if args.warmup > 0 and wl["grid"]["ndim"] == 3:
        # the 3-D box is statistically stationary: warm up on the timed instance
        sim.step(args.warmup)
        sim.sync()
    step0 = sim.diag()["step"]
    if not args.no_kernel_timing:
        # the particle kernel (the roofline's kernel) is timed inside the timed
        # region; the other kernels only afterwards (each timed kernel adds a
        # few microseconds between launches)
        sim.timing_enable("particles")
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.sync()
    wall = t1 - t0
    _, _, pushed = sim.history(step0, args.steps)
    total = int(pushed.sum())
    value = total / wall
    timing = sim.timing() if not args.no_kernel_timing else {}
    d = sim.diag()
    breakdown = {}
    if not args.no_kernel_timing:
        # per-kernel breakdown over a short window after the timed region
        sim.timing_enable(True)
        sim.step(min(64, max(1, args.steps // 4)))
        breakdown = {k: round(v[0] / max(v[1], 1), 4) for k, v in sim.timing().items()}

    roof = None
    if timing:
        ms, launches = timing["particles"]
        avg_s = ms / 1e3 / max(launches, 1)
        ndim = wl["grid"]["ndim"]
        per_launch_bytes = BYTES_PER_PARTICLE_STEP[(ndim, args.precision)] * total / max(launches, 1)
        achieved = per_launch_bytes / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": _measured_traffic(args.precision, args.workload),
                "kernel": "k_particles2d" if wl["grid"]["ndim"] == 2 else "k_particles3d",
                "algorithmic_bytes_per_launch": per_launch_bytes,
                "particle_kernel_ms_per_launch": round(avg_s * 1e3, 4),
                "kernel_ms_per_launch_after_timed_region": breakdown}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "steps_timed": args.steps,
                   "particles_start": int(wl["w"].size), "particles_end": int(d["particles"]),
                   "occupancy_max_end": d["occupancy_max"], "relayouts": d["relayouts"]},
        "roofline": roof,
    }
    if copy_cal:
        out["copy_calibration"] = copy_cal
    sim.close()
    del sim
    if args.scan > 0:
        print(f"[bench] batched scan of {args.scan} simulations", file=sys.stderr, flush=True)
        out["batched_scan"] = _scan_bench(args.scan, args.scan_steps, args.precision)
    if args.serve > 0:
        lo, hi = (int(v) for v in args.serve_steps.split(","))
        print(f"[bench] serving {args.serve} requests", file=sys.stderr, flush=True)
        out["served_scan"] = _serve_bench(args.serve, args.serve_rate, (lo, hi), 200.0,
                                          args.precision)
    if not args.no_cpu:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = _cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
