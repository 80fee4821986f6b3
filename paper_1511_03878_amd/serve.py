"""Serving loop for parameter-scan simulations: continuous batching on one GPU.

Requests (independent 2-D laser-wakefield simulations of uneven size) arrive
over time.  The server admits a request as soon as its estimated device
memory fits the remaining HBM budget, adds it to one `Batch` -- a single work
queue, one persistent particle launch and one Yee / re-binning pass per step
cover every resident simulation -- and advances the batch in short slices.
Simulations that finish their step budget are read back, removed and their
memory released; requests that arrived meanwhile are admitted at the next
slice boundary.  Time-to-result is completion minus arrival (queueing
included).

All stepping runs in libpic.so; this module only schedules.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Optional

import numpy as np

from . import workloads as W
from .sim import Batch, Sim, estimate_bytes


@dataclasses.dataclass
class Request:
    rid: int
    params: dict            # a draw of workloads.scan_params
    nsteps: int
    arrival: float          # seconds after the start of the run
    admitted: Optional[float] = None
    done: Optional[float] = None
    result: Optional[dict] = None
    nparticles: int = 0
    bytes: int = 0
    workload: Optional[dict] = dataclasses.field(default=None, repr=False)

    @property
    def time_to_result(self) -> float:
        return self.done - self.arrival


def make_workload(req: Request, seed: int = W.DEFAULT_SEED, patch=(32, 32)):
    return W.scan_sim(req.params, seed=seed + req.rid, patch=tuple(patch))


def particle_count(wl: dict) -> int:
    """Particles a workload loads (for admission before the simulation
    exists): explicit arrays, or a uniform or ramp species description (ppc in
    every cell at or beyond the ramp start)."""
    if "x" in wl:
        return int(np.asarray(wl["w"]).size)
    sp, g = wl["species"], wl["grid"]
    cells = int(np.prod(g["n"]))
    if sp["profile"] == "uniform":
        return sp["ppc"] * cells
    if sp["profile"] == "ramp":
        X0 = sp["param"][0] / g["d"][0]
        cols = int(np.count_nonzero(np.arange(g["n"][0]) >= X0))
        return sp["ppc"] * cols * (cells // g["n"][0])
    raise ValueError("admission estimate needs explicit arrays or a uniform / ramp species")


def default_result(sim: Sim) -> dict:
    """What a finished request returns: diagnostics, energy history and fields."""
    d = sim.diag()
    U, K, P = sim.history(max(0, d["step"] - min(d["step"], 4096)), min(d["step"], 4096))
    return {"diag": d, "U": U, "K": K, "pushed": P,
            "Ey": sim.field("Ey"), "Ex": sim.field("Ex"), "Bz": sim.field("Bz")}


class Server:
    """Admits requests against an HBM budget and steps them together."""

    def __init__(self, budget_bytes: int, precision: int = 32, slice_steps: int = 25,
                 result_fn: Callable[[Sim], dict] = default_result, clock=time.perf_counter,
                 max_members: int = 256, patch=(32, 32), tune: Optional[dict] = None):
        self.budget = int(budget_bytes)
        self.precision = precision
        self.slice_steps = slice_steps
        self.result_fn = result_fn
        self.clock = clock
        self.max_members = max_members
        self.patch = tuple(patch)       # patch edge of every request (e.g. from the patch tuner)
        self.tune = dict(tune or {})    # descriptor settings of every request
        self.batch = Batch(precision)
        self.in_use = 0
        self.peak_in_use = 0
        self.charges = []          # (resident count, bytes charged, bytes the residents hold)
        self.resident: dict = {}   # sim handle -> (Request, Sim)
        self._t0 = clock()
        self._skew = 0.0

    def _admit(self, req: Request, now: float) -> bool:
        if req.workload is None:
            req.workload = make_workload(req, patch=self.patch)
            wl = req.workload
            req.nparticles = particle_count(wl)
            req.bytes = estimate_bytes(wl["grid"], self.precision, req.nparticles, **self.tune)
        wl = req.workload
        if req.bytes > self.budget:
            raise ValueError(f"request {req.rid} needs {req.bytes} B, above the whole budget")
        if self.in_use + req.bytes > self.budget or len(self.resident) >= self.max_members:
            return False
        sim = Sim.from_workload(wl, precision=self.precision, **self.tune)
        req.nparticles = sim.num_particles()
        req.workload = None  # the state lives on the GPU now
        self.batch.add(sim, req.nsteps)
        self.resident[sim.handle.value] = (req, sim)
        self._charge()
        req.admitted = now
        return True

    def _charge(self):
        """Charge every resident simulation the device memory it holds now
        (capacity growth after an overflowing patch raises it), but at least
        its admission estimate."""
        held = [sim.device_bytes() for _, sim in self.resident.values()]
        self.in_use = sum(max(req.bytes, h) for (req, _), h in zip(self.resident.values(), held))
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        self.charges.append((len(held), self.in_use, sum(held)))

    def _retire(self, now: float):
        for sim in self.batch.finished():
            req, _ = self.resident.pop(sim.handle.value)
            req.result = self.result_fn(sim)
            req.done = self._now()
            self.batch.remove(sim)
            sim.close()
        self._charge()

    def _now(self) -> float:
        return self.clock() - self._t0 + self._skew

    def run(self, requests, realtime: bool = True, warmup: int = 0) -> dict:
        """Serve `requests` (arrival times in seconds from now).  With
        realtime=False, idle gaps before the next arrival are skipped (the
        clock jumps ahead) instead of slept through.  The first `warmup`
        requests (by arrival) are served but left out of the time-to-result
        percentiles."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        waiting = collections.deque()
        i = 0
        self._t0 = self.clock()
        self._skew = 0.0
        slices = 0
        while i < len(reqs) or waiting or self.resident:
            now = self._now()
            while i < len(reqs) and reqs[i].arrival <= now:
                waiting.append(reqs[i])
                i += 1
            while waiting and self._admit(waiting[0], now):
                waiting.popleft()
            if not self.resident:
                if waiting:
                    raise RuntimeError("a waiting request can never be admitted")
                if i < len(reqs):
                    gap = reqs[i].arrival - now
                    if gap > 0:
                        if realtime:
                            time.sleep(gap)
                        else:
                            self._skew += gap
                continue
            self.batch.step(self.slice_steps)
            slices += 1
            self._retire(now)
        wall = self._now()
        meas = reqs[warmup:] if warmup < len(reqs) else reqs
        ttr = np.array([r.time_to_result for r in meas])
        psteps = sum(r.nparticles * r.nsteps for r in reqs)
        return {"requests": len(meas), "wall_s": wall, "particle_steps": psteps,
                "throughput": psteps / wall if wall > 0 else 0.0,
                "ttr_p50_s": float(np.percentile(ttr, 50)), "ttr_p99_s": float(np.percentile(ttr, 99)),
                "ttr_max_s": float(ttr.max()), "slices": slices, "peak_in_use_bytes": self.peak_in_use}


def make_requests(count: int, rate: float, steps_range=(200, 2000), seed: int = W.DEFAULT_SEED,
                  scan_patch: int = 32):
    """Poisson arrivals of scan simulations with step counts uniform in steps_range."""
    params = W.scan_params(count, seed=seed, patch=scan_patch)
    arrivals = W.poisson_arrivals(count, rate, seed=seed)
    g = W.rng(seed, W.STREAM_SCAN + 10)
    steps = g.integers(steps_range[0], steps_range[1] + 1, size=count)
    return [Request(rid=k, params=params[k], nsteps=int(steps[k]), arrival=float(arrivals[k]))
            for k in range(count)]
