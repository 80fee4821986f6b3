"""Seeded synthetic workload descriptions (inputs only; none of the method's arithmetic).

A workload is a grid description, a species description (density profile,
loading rule, particles per cell, temperature, seed) and, for the
laser-wakefield boxes, a laser description (a0, waist, duration, focus).  The
library (pic_species_add, pic_particles_init, pic_laser_add) and the oracle
each turn a description into particles and an incident field with their own
code; this module only states the parameters, and draws the parameters of the
batched and served scans.

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
                  sphere (particle count proportional to density);
  scan_params  -- the parameter draws of the batched / served scans.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULT_SEED = 151103878
ME_C2_KEV = 510.99895  # electron rest energy, keV

# random-number streams of one seed: 0 and 1 are the particle loaders'
# (positions, momenta); 2 and 3 are drawn here with numpy
STREAM_SCAN, STREAM_ARRIVAL = 2, 3
PROFILES = {"uniform": 0, "ramp": 1, "cos_sphere": 2}
LOADINGS = {"weight": 0, "count": 1}


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def cfl_dt(d, factor: float = 0.95) -> float:
    """Time step as a fraction of the Yee stability limit (sum 1/d^2)^(-1/2)."""
    return factor / math.sqrt(sum(1.0 / (x * x) for x in d))


def temperature(T_keV: float) -> float:
    """kT / (m c^2) of electrons at T_keV."""
    return T_keV / ME_C2_KEV


def species(profile: str, ppc: int, n0: float = 1.0, loading: str = "weight", param=(),
            T_keV: float = 0.0, seed: int = DEFAULT_SEED, q: float = -1.0, m: float = 1.0) -> dict:
    """Species description (see pic_species_add): profile 'uniform', 'ramp'
    (param = x0, x1) or 'cos_sphere' (param = modulation, centre x, y, z,
    radius, factor), loading 'weight' (ppc per plasma cell, weight n / ppc) or
    'count' (round(ppc n / n0) per cell, weight n0 / ppc)."""
    p = [float(v) for v in param] + [0.0] * (6 - len(param))
    return dict(profile=profile, loading=loading, ppc=int(ppc), n0=float(n0), param=p,
                temperature=temperature(T_keV), seed=int(seed), q=float(q), m=float(m))


def gaussian_laser(a0, w0, tau, t0, x_focus, y_center, omega0=1.0, phase=0.0, polarisation=1) -> dict:
    """Laser description (see pic_laser_add)."""
    return dict(a0=float(a0), omega0=float(omega0), w0=float(w0), tau=float(tau), t0=float(t0),
                x_focus=float(x_focus), y_center=float(y_center), phase=float(phase),
                polarisation=int(polarisation))


def uniform_2d(n=(128, 128), d=(0.1, 0.1), patch=(16, 16), ppc=16, n0=1.0,
               T_keV=1.0, seed=DEFAULT_SEED, cfl=0.95):
    """Thermal periodic 2D3V box: one electron species, immobile neutralising
    ions (they enter only the Gauss diagnostic), omega_p units."""
    grid = dict(ndim=2, n=[int(v) for v in n], d=list(d), dt=cfl_dt(d, cfl), patch=list(patch),
                periodic=[1, 1], q=-1.0, m=1.0)
    return dict(name="uniform_2d", grid=grid, species=species("uniform", ppc, n0, T_keV=T_keV, seed=seed),
                laser=None)


def lwfa_2d(n=(4096, 1024), lam=2.0 * math.pi, cells_per_lam=(32, 8), patch=(32, 32),
            ppc=4, n_plateau=0.003, ramp=(2.0, 12.0), a0=4.0, w0_lam=12.0,
            tau_lam=9.375, seed=DEFAULT_SEED, cfl=0.95, y_center=None):
    """2D3V laser-wakefield box in laser units (omega_0 = 1, lambda = 2 pi).

    Vacuum for x < ramp[0] lambda, a linear density ramp up to ramp[1] lambda,
    then a plateau at n_plateau n_c; ppc electrons per plasma cell with
    weights proportional to the local density; cold.  Open x faces (the laser
    is driven through x = 0, particles are absorbed), periodic y.  The laser:
    y-polarised, waist w0_lam lambda focused at the ramp start, intensity FWHM
    tau_lam lambda / c, envelope peak at t0 = 2 tau.
    """
    n = tuple(int(v) for v in n)
    d = (lam / cells_per_lam[0], lam / cells_per_lam[1])
    x0, x1 = ramp[0] * lam, ramp[1] * lam
    tau = tau_lam * lam
    laser = gaussian_laser(a0, w0_lam * lam, tau, 2.0 * tau, x_focus=x0,
                           y_center=n[1] * d[1] / 2 if y_center is None else y_center)
    grid = dict(ndim=2, n=list(n), d=list(d), dt=cfl_dt(d, cfl), patch=list(patch),
                periodic=[0, 1], q=-1.0, m=1.0)
    # density of every cell column at its centre, for a moving window's
    # injection (the plateau continues beyond the table)
    X0, X1 = x0 / d[0], x1 / d[0]
    cc = np.arange(int(math.ceil(X1)) + 2) + 0.5
    col_dens = np.where(cc < X0, 0.0, np.where(cc >= X1, n_plateau, n_plateau * (cc - X0) / (X1 - X0)))
    return dict(name="lwfa_2d", grid=grid, laser=laser, column_density=col_dens, ppc=ppc,
                species=species("ramp", ppc, n_plateau, param=(x0, x1), seed=seed))


def lwfa_2d_small(seed=DEFAULT_SEED, n=(512, 128), patch=(32, 32), **kw):
    """The LWFA box at a size the oracle finishes in seconds: same cell sizes,
    ramp and laser shape, a narrower waist so the beam fits the box."""
    args = dict(n=n, patch=patch, ramp=(1.0, 3.0), w0_lam=n[1] / 8 / 6.0, tau_lam=2.0,
                a0=4.0, seed=seed)
    args.update(kw)
    out = lwfa_2d(**args)
    out["name"] = "lwfa_2d_small"
    return out


def blob_3d(n=(512, 256, 256), d=(0.1, 0.1, 0.1), patch=(16, 16, 16), ppc0=8, n0=1.0,
            mod=0.9, blob_radius=20.0, blob_factor=4.0, T_keV=10.0, seed=DEFAULT_SEED,
            cfl=0.95):
    """3D3V periodic box: density n0 (1 + mod cos(k x)), k = 2 pi / L_x, plus
    an over-dense sphere (blob_factor n0, radius blob_radius cells) at the box
    centre; round(ppc0 n / n0) particles per cell with constant weight
    n0 / ppc0; thermal."""
    n = tuple(int(v) for v in n)
    centre = [n[a] * d[a] / 2 for a in range(3)]
    grid = dict(ndim=3, n=list(n), d=list(d), dt=cfl_dt(d, cfl), patch=list(patch),
                periodic=[1, 1, 1], q=-1.0, m=1.0)
    sp = species("cos_sphere", ppc0, n0, loading="count",
                 param=(mod, *centre, blob_radius * d[0], blob_factor), T_keV=T_keV, seed=seed)
    return dict(name="blob_3d", grid=grid, species=sp, laser=None)


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


def scan_sim(p, seed=DEFAULT_SEED, patch=(32, 32)):
    """One scan member: the LWFA box with the drawn parameters, waist L_y / 6,
    tau = 4 lambda/c, vacuum x < 1 lambda, ramp 1 -> 3 lambda."""
    ny_lam = p["n"][1] / 8.0
    out = lwfa_2d(n=p["n"], patch=patch, ppc=p["ppc"], n_plateau=p["n_plateau"],
                  ramp=(1.0, 3.0), a0=p["a0"], w0_lam=ny_lam / 6.0, tau_lam=4.0, seed=seed)
    out["name"] = "scan_2d"
    return out


def poisson_arrivals(count, rate, seed=DEFAULT_SEED):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    g = rng(seed, STREAM_ARRIVAL)
    return np.cumsum(g.exponential(1.0 / rate, size=count))
