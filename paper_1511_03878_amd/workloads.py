"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

This module is the single source of inputs for both the HIP path and the
oracle.  It builds grid descriptions, particle arrays (cell-unit positions,
momenta u = p/(m c), weights) and the incident-field table that drives the
x = 0 face.  It imports nothing else from the package.

Units: c = eps0 = e = m_e = 1, lengths in c/omega_r, time in 1/omega_r,
densities in n_r = eps0 m_e omega_r^2 / e^2 (so the critical density n_c = 1
when omega_r is the laser frequency).  The paper quotes resolutions in these
units (section 2.2).

Workloads (their shapes follow the paper's LWFA and load-imbalance regimes,
sections 2.2, 3 and 3.1; the paper publishes no input data, so every input is
synthetic and seeded):
  uniform_2d   -- thermal periodic box (the 128 x 128, 16 ppc, 1 keV case);
  lwfa_2d      -- laser-wakefield box: Gaussian laser driven through x = 0,
                  cold electrons behind a linear density ramp, open x faces;
  blob_3d      -- 3-D periodic box with a modulated density and an over-dense
                  sphere (ppc proportional to density);
  scan_params  -- the parameter draws of the batched / served scans.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULT_SEED = 151103878
ME_C2_KEV = 510.99895  # electron rest energy, keV

# random-number streams of one seed
STREAM_POS, STREAM_MOM, STREAM_SCAN, STREAM_ARRIVAL = 0, 1, 2, 3


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def cfl_dt(d, factor: float = 0.95) -> float:
    """Time step as a fraction of the Yee stability limit (sum 1/d^2)^(-1/2)."""
    return factor / math.sqrt(sum(1.0 / (x * x) for x in d))


def thermal_sigma(T_keV: float) -> float:
    """Per-component momentum spread sqrt(T / m c^2) of a non-relativistic Maxwellian."""
    return math.sqrt(T_keV / ME_C2_KEV)


# ---------------------------------------------------------------------------
# particle loading

def _cells_and_offsets(n, ppc_of_cell, g):
    """Cell coordinates (row-major, x fastest) repeated ppc times, plus
    uniform in-cell offsets; returns positions in cell units."""
    nd = len(n)
    ncell = int(np.prod(n))
    ppc = np.broadcast_to(np.asarray(ppc_of_cell, dtype=np.int64), (ncell,))
    cell = np.repeat(np.arange(ncell, dtype=np.int64), ppc)
    coords = []
    rem = cell
    for a in range(nd):
        coords.append(rem % n[a])
        rem = rem // n[a]
    pos = [coords[a].astype(np.float64) + g.random(cell.size) for a in range(nd)]
    # an offset of exactly 1.0 cannot occur (random() is in [0, 1)), but the
    # addition can round up to the next cell for huge n; keep positions in range
    for a in range(nd):
        np.minimum(pos[a], np.nextafter(float(n[a]), 0.0), out=pos[a])
    return pos


def uniform_2d(n=(128, 128), d=(0.1, 0.1), patch=(16, 16), ppc=16, n0=1.0,
               T_keV=1.0, seed=DEFAULT_SEED, cfl=0.95):
    """Thermal periodic 2D3V box: one electron species, immobile neutralising
    ions (they enter only the Gauss diagnostic), omega_p units."""
    n = tuple(int(v) for v in n)
    g_pos = rng(seed, STREAM_POS)
    g_mom = rng(seed, STREAM_MOM)
    pos = _cells_and_offsets(n, ppc, g_pos)
    npart = pos[0].size
    sig = thermal_sigma(T_keV)
    mom = [sig * g_mom.standard_normal(npart) for _ in range(3)]
    w = np.full(npart, n0 / ppc)
    grid = dict(ndim=2, n=list(n), d=list(d), dt=cfl_dt(d, cfl), patch=list(patch),
                periodic=[1, 1], q=-1.0, m=1.0)
    return dict(name="uniform_2d", grid=grid, x=pos, u=mom, w=w, laser=None)


def gaussian_beam_2d(ny, dy, dt, nsteps, a0, w0, tau, t0, x_focus, y_center,
                     omega0=1.0, phase=0.0):
    """Incident Ey at the x = 0 face for a y-polarised 2-D Gaussian beam.

    Row t is the field at time (t + 1/2) dt on the Ey positions y = (j + 1/2) dy.
    Envelope exp(-2 ln2 (t - t0)^2 / tau^2) (tau = intensity FWHM); 2-D
    paraxial beam (waist w0 at x_focus): amplitude sqrt(w0 / w(x)), Gouy phase
    arctan(x / x_R) / 2, wavefront curvature; peak field a0 * omega0.
    """
    xr = 0.5 * omega0 * w0 * w0
    xi = 0.0 - x_focus
    wx = w0 * math.sqrt(1.0 + (xi / xr) ** 2)
    inv_r = xi / (xi * xi + xr * xr)
    gouy = 0.5 * math.atan2(xi, xr)
    y = (np.arange(ny) + 0.5) * dy - y_center
    t = (np.arange(nsteps) + 0.5) * dt
    amp = a0 * omega0 * math.sqrt(w0 / wx)
    trans = np.exp(-(y / wx) ** 2)
    env = np.exp(-2.0 * math.log(2.0) * ((t - t0) / tau) ** 2)
    ph = omega0 * (t[:, None] - t0) - 0.5 * omega0 * y[None, :] ** 2 * inv_r + gouy + phase
    return amp * env[:, None] * trans[None, :] * np.sin(ph)


def lwfa_2d(n=(4096, 1024), lam=2.0 * math.pi, cells_per_lam=(32, 8), patch=(32, 32),
            ppc=4, n_plateau=0.003, ramp=(2.0, 12.0), a0=4.0, w0_lam=12.0,
            tau_lam=9.375, nsteps=2000, seed=DEFAULT_SEED, cfl=0.95, y_center=None):
    """2D3V laser-wakefield box in laser units (omega_0 = 1, lambda = 2 pi).

    Vacuum for x < ramp[0] lambda, a linear density ramp up to ramp[1] lambda,
    then a plateau at n_plateau n_c; ppc electrons per plasma cell with
    weights proportional to the local density; cold.  Open x faces (the laser
    is driven through x = 0, particles are absorbed), periodic y.
    """
    n = tuple(int(v) for v in n)
    d = (lam / cells_per_lam[0], lam / cells_per_lam[1])
    dt = cfl_dt(d, cfl)
    x0 = ramp[0] * lam / d[0]  # cell units
    x1 = ramp[1] * lam / d[0]
    ppc_cell = np.zeros(n[0] * n[1], dtype=np.int64)
    plasma_col = (np.arange(n[0]) + 1) > x0  # cells that reach into the plasma
    ppc_cell.reshape(n[1], n[0])[:, plasma_col] = ppc
    g_pos = rng(seed, STREAM_POS)
    pos = _cells_and_offsets(n, ppc_cell, g_pos)
    xs = pos[0]
    keep = xs >= x0
    pos = [p[keep] for p in pos]
    xs = pos[0]
    dens = np.where(xs >= x1, n_plateau, n_plateau * (xs - x0) / (x1 - x0))
    w = dens / ppc
    npart = w.size
    mom = [np.zeros(npart) for _ in range(3)]
    Ly = n[1] * d[1]
    w0 = w0_lam * lam
    tau = tau_lam * lam
    laser_ey = gaussian_beam_2d(n[1], d[1], dt, nsteps, a0, w0, tau, 2.0 * tau,
                                x_focus=ramp[0] * lam,
                                y_center=Ly / 2 if y_center is None else y_center)
    grid = dict(ndim=2, n=list(n), d=list(d), dt=dt, patch=list(patch),
                periodic=[0, 1], q=-1.0, m=1.0)
    # density of every cell column at its centre, for a moving window's
    # injection (the plateau continues beyond the table)
    cc = np.arange(int(math.ceil(x1)) + 2) + 0.5
    col_dens = np.where(cc < x0, 0.0, np.where(cc >= x1, n_plateau, n_plateau * (cc - x0) / (x1 - x0)))
    return dict(name="lwfa_2d", grid=grid, x=pos, u=mom, w=w,
                laser=dict(ey=laser_ey, ez=None), column_density=col_dens, ppc=ppc)


def lwfa_2d_small(nsteps=200, seed=DEFAULT_SEED, n=(512, 128), patch=(32, 32), **kw):
    """The LWFA box at a size the oracle finishes in seconds: same cell sizes,
    ramp and laser shape, a narrower waist so the beam fits the box."""
    args = dict(n=n, patch=patch, ramp=(1.0, 3.0), w0_lam=n[1] / 8 / 6.0, tau_lam=2.0,
                a0=4.0, nsteps=nsteps, seed=seed)
    args.update(kw)
    out = lwfa_2d(**args)
    out["name"] = "lwfa_2d_small"
    return out


def blob_3d(n=(512, 256, 256), d=(0.1, 0.1, 0.1), patch=(16, 16, 16), ppc0=8, n0=1.0,
            mod=0.9, blob_radius=20.0, blob_factor=4.0, T_keV=10.0, seed=DEFAULT_SEED,
            cfl=0.95):
    """3D3V periodic box: density n0 (1 + mod cos(k x)), k = 2 pi / L_x, plus
    an over-dense sphere (blob_factor n0) at the box centre; ppc proportional
    to density (round(ppc0 n / n0)) with constant weight n0 / ppc0; thermal."""
    n = tuple(int(v) for v in n)
    ic = [np.arange(v) + 0.5 for v in n]
    dens_x = n0 * (1.0 + mod * np.cos(2.0 * math.pi * ic[0] / n[0]))
    Z, Y, X = np.meshgrid(ic[2], ic[1], ic[0], indexing="ij")
    r2 = (X - n[0] / 2) ** 2 + (Y - n[1] / 2) ** 2 + (Z - n[2] / 2) ** 2
    dens = np.broadcast_to(dens_x[None, None, :], r2.shape).copy()
    dens[r2 <= blob_radius ** 2] = blob_factor * n0
    ppc_cell = np.rint(ppc0 * dens / n0).astype(np.int64).reshape(-1)
    del X, Y, Z, r2, dens
    g_pos = rng(seed, STREAM_POS)
    g_mom = rng(seed, STREAM_MOM)
    pos = _cells_and_offsets(n, ppc_cell, g_pos)
    npart = pos[0].size
    sig = thermal_sigma(T_keV)
    mom = [sig * g_mom.standard_normal(npart) for _ in range(3)]
    w = np.full(npart, n0 / ppc0)
    grid = dict(ndim=3, n=list(n), d=list(d), dt=cfl_dt(d, cfl), patch=list(patch),
                periodic=[1, 1, 1], q=-1.0, m=1.0)
    return dict(name="blob_3d", grid=grid, x=pos, u=mom, w=w, laser=None)


def cold_wave_2d(n=(64, 8), d=(0.1, 0.1), patch=(16, 8), ppc_side=(2, 2), n0=1.0,
                 amp=1e-3, cfl=0.95):
    """Cold plasma on a regular lattice with a sinusoidal velocity perturbation
    u_x = amp sin(2 pi x / L_x): with fields and charge initially balanced it
    excites a Langmuir oscillation at omega_p (omega_p units)."""
    nx, ny = n
    px, py = ppc_side
    xs = (np.arange(nx * px) + 0.5) / px
    ys = (np.arange(ny * py) + 0.5) / py
    Y, X = np.meshgrid(ys, xs, indexing="ij")
    X = X.reshape(-1)
    Y = Y.reshape(-1)
    npart = X.size
    w = np.full(npart, n0 / (px * py))
    mom = [amp * np.sin(2.0 * math.pi * X / nx), np.zeros(npart), np.zeros(npart)]
    grid = dict(ndim=2, n=[nx, ny], d=list(d), dt=cfl_dt(d, cfl), patch=list(patch),
                periodic=[1, 1], q=-1.0, m=1.0)
    return dict(name="cold_wave_2d", grid=grid, x=[X, Y], u=mom, w=w, laser=None)


def scan_params(count=64, seed=DEFAULT_SEED, patch=32):
    """Parameter draws of the batched / served scans: grid log-uniform in
    [256, 2048] x [128, 512] (rounded to the patch size), density uniform in
    [0.001, 0.01] n_c, a0 uniform in [1, 6], ppc uniform in {2..8}."""
    g = rng(seed, STREAM_SCAN)
    out = []
    for _ in range(count):
        nx = int(round(math.exp(g.uniform(math.log(256), math.log(2048))) / patch)) * patch
        ny = int(round(math.exp(g.uniform(math.log(128), math.log(512))) / patch)) * patch
        out.append(dict(n=(max(nx, patch), max(ny, patch)),
                        n_plateau=float(g.uniform(0.001, 0.01)),
                        a0=float(g.uniform(1.0, 6.0)),
                        ppc=int(g.integers(2, 9))))
    return out


def scan_sim(p, nsteps, seed=DEFAULT_SEED, patch=(32, 32)):
    """One scan member: the LWFA box with the drawn parameters, waist L_y / 6,
    tau = 4 lambda/c, vacuum x < 1 lambda, ramp 1 -> 3 lambda."""
    ny_lam = p["n"][1] / 8.0
    out = lwfa_2d(n=p["n"], patch=patch, ppc=p["ppc"], n_plateau=p["n_plateau"],
                  ramp=(1.0, 3.0), a0=p["a0"], w0_lam=ny_lam / 6.0, tau_lam=4.0,
                  nsteps=nsteps, seed=seed)
    out["name"] = "scan_2d"
    return out


def poisson_arrivals(count, rate, seed=DEFAULT_SEED):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    g = rng(seed, STREAM_ARRIVAL)
    return np.cumsum(g.exponential(1.0 / rate, size=count))


def to_float32_state(wl):
    """The workload rounded to what an FP32 run stores, promoted back to FP64.

    Positions are stored as FP32 offsets from their patch origin (patches of
    at most 2^k cells), so they are truncated to multiples of 2^-(24-k): then
    every offset is exact in FP32 and the FP64 global value is exact too.
    Momenta and weights are rounded to FP32.  An FP64 reference started from
    this state sees exactly the initial state the FP32 path holds."""
    out = dict(wl)
    pmax = max(wl["grid"]["patch"])
    k = max(1, int(math.ceil(math.log2(pmax))))
    q = 2.0 ** -(24 - k)
    out["x"] = [np.floor(np.asarray(a, dtype=np.float64) / q) * q for a in wl["x"]]
    out["u"] = [np.asarray(a, dtype=np.float32).astype(np.float64) for a in wl["u"]]
    out["w"] = np.asarray(wl["w"], dtype=np.float32).astype(np.float64)
    return out
