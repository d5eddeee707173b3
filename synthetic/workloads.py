"""Seeded workload recipes: grids, fields, ensembles of injected electrons.

The paper injects 81 keV electrons at r = 0.28 AU and 24 deg latitude with a
mean free path of 0.1, 0.5 or 1 AU (Sect. 3).  The recipes below keep those
values and add the spreads of the synthetic benchmark workloads: longitude
uniform in +-2 deg, pitch-angle cosine uniform in [0, 1].

An ``Ensemble`` is a plain description; both the oracle and the HIP library
take its numbers as arguments.  Injection itself (drawing positions, pitch
cosines, free paths from the counter-based generator) is done by each side.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Callable, List

import numpy as np

from .constants import AU, E_CHARGE, M_ELECTRON, KEV, C_LIGHT
from .grid import SphericalGrid
from . import fields

HOUR = 3600.0


@dataclass
class Ensemble:
    n: int                      # electrons in this ensemble
    ensemble: int               # ensemble index (second word of the generator key)
    seed: int                   # first word of the generator key
    ekin: float = 81.0 * KEV    # J
    r0: float = 0.28 * AU       # m
    lat0: float = math.radians(24.0)
    lon0: float = 0.0
    dlon: float = math.radians(2.0)     # longitude half-width
    dr0: float = 0.0                    # radial half-width
    dlat: float = 0.0                   # latitude half-width
    mu_lo: float = 0.0                  # pitch-angle cosine range at injection
    mu_hi: float = 1.0
    lambda_par: float = 0.5 * AU        # m; <= 0 disables scattering
    r_in: float = 0.28 * AU
    r_out: float = 1.97 * AU
    max_steps: int = 0                  # 0: no stop
    q: float = -E_CHARGE
    m: float = M_ELECTRON
    drift_free: bool = False
    scatter_law: int = 0                # 0: mu' = 1 - 2a ; 1: mu' = +-sqrt(a)
    rebirth_steps: int = 0              # > 0: an exit before this step count is a rebirth
    v_wind: float = 0.0                 # > 0: scattering centres move with a radial wind of this speed (m/s)


@dataclass
class Workload:
    name: str
    grid: SphericalGrid
    build_field: Callable            # (grid, device) -> float64 [nr][nth][nph][12]
    ensembles: List[Ensemble]
    dt: float
    n_steps: int
    store_dtype: str = "f64"         # field storage on the device
    bin_interval: int = 64

    @property
    def n_particles(self) -> int:
        return sum(e.n for e in self.ensembles)


def gamma_of(ekin: float, m: float = M_ELECTRON) -> float:
    return 1.0 + ekin / (m * C_LIGHT ** 2)


def r_out_default(grid: SphericalGrid) -> float:
    """Outer exit radius one cell inside the grid, so the predictor stays in the stencil."""
    return grid.r_max - grid.dr


def config_small(seed: int = 0, n: int = 1024, hours: float = 2.0, store_dtype: str = "f64") -> Workload:
    """1,024 electrons at 81 keV, analytic Parker spiral on a 64x32x64 grid over
    [0.1, 2] AU, lambda = 0.5 AU, dt = 1 s, 2 h."""
    grid = SphericalGrid(64, 32, 64, 0.1 * AU, 2.0 * AU)
    ens = Ensemble(n=n, ensemble=0, seed=seed, lambda_par=0.5 * AU, r_in=0.28 * AU,
                   r_out=r_out_default(grid))
    return Workload("parker-64x32x64-1k", grid, lambda g, device=None: fields.parker(g, device),
                    [ens], 1.0, int(round(hours * HOUR)), store_dtype)


def config_paper_scale(seed: int = 0, n: int = 1 << 20, hours: float = 24.0, field_seed: int = 1,
                       store_dtype: str = "f32") -> Workload:
    """1M electrons at 81 keV split over lambda in {0.1, 0.5, 1.0} AU, Parker
    spiral plus 16 seeded Fourier modes (dB/B = 0.1, |k| in [2, 20]/AU) on a
    256x128x256 grid over [0.1, 2] AU, dt = 1 s, 24 h, binning every 64 steps."""
    grid = SphericalGrid(256, 128, 256, 0.1 * AU, 2.0 * AU)
    lams = (0.1 * AU, 0.5 * AU, 1.0 * AU)
    counts = [n // 3 + (1 if i < n % 3 else 0) for i in range(3)]
    ens = [Ensemble(n=c, ensemble=i, seed=seed, lambda_par=lam, r_in=0.28 * AU,
                    r_out=r_out_default(grid)) for i, (c, lam) in enumerate(zip(counts, lams))]
    return Workload("parker+16modes-256x128x256-1M", grid,
                    lambda g, device=None: fields.perturbed_parker(g, field_seed, device=device),
                    ens, 1.0, int(round(hours * HOUR)), store_dtype, 64)


def config_steady(seed: int = 0, n: int = 1000, hours: float = 150.0, dt: float = 0.54, field_seed: int = 1,
                  lambda_au: float = 0.5, store_dtype: str = "f32") -> Workload:
    """Steady-state run of Sect. 3: 10^3 electrons of 81 keV released with pitch
    angle 0 at 0.28 AU and 24 deg latitude, all on one field line, lambda = 0.5 AU,
    dt = 0.54 s, reborn at once whenever they leave the shell, for 150 h.  The
    field is the paper-scale one (Parker spiral plus 16 Fourier modes on
    256x128x256 over [0.1, 2] AU); its radial extent puts the outer exit shell
    just inside 2 AU, the paper's value for its lambda = 0.1 AU run."""
    grid = SphericalGrid(256, 128, 256, 0.1 * AU, 2.0 * AU)
    n_steps = int(round(hours * HOUR / dt))
    ens = Ensemble(n=n, ensemble=0, seed=seed, r0=0.28 * AU, lat0=math.radians(24.0), lon0=0.0, dlon=0.0,
                   mu_lo=1.0, mu_hi=1.0, lambda_par=lambda_au * AU, r_in=0.28 * AU, r_out=r_out_default(grid),
                   rebirth_steps=n_steps)
    return Workload(f"steady-{n}e-{hours:g}h", grid,
                    lambda g, device=None: fields.perturbed_parker(g, field_seed, device=device),
                    [ens], dt, n_steps, store_dtype, 100)


def config_batched(seed: int = 0, n_ens: int = 64, total: int = 4 << 20, field_seed: int = 1,
                   dt: float = 1.0, store_dtype: str = "f32", grid: SphericalGrid = None,
                   hours_lo: float = 6.0, hours_hi: float = 48.0) -> Workload:
    """64 ensembles of log-uniform size in [1k, 256k] summing to 4M; energies
    log-uniform 20-300 keV, lambda log-uniform 0.05-2 AU, r0 in [0.2, 0.4] AU,
    latitude in +-40 deg, longitude uniform, stop times uniform in 6-48 h."""
    rng = np.random.default_rng(1000 + seed)
    grid = grid or SphericalGrid(256, 128, 256, 0.1 * AU, 2.0 * AU)
    lo, hi = min(1 << 10, total // n_ens), min(1 << 18, total)
    w = np.exp(rng.uniform(math.log(lo), math.log(hi), n_ens))
    # rescale towards the requested total while respecting [lo, hi]
    for _ in range(100):
        s = total / w.sum()
        w = np.clip(w * s, lo, hi)
        if abs(w.sum() - total) < 1:
            break
    counts = np.floor(w).astype(np.int64)
    counts[np.argmax(counts < hi)] += total - counts.sum()
    ekin = np.exp(rng.uniform(math.log(20.0), math.log(300.0), n_ens)) * KEV
    lam = np.exp(rng.uniform(math.log(0.05), math.log(2.0), n_ens)) * AU
    r0 = rng.uniform(0.2, 0.4, n_ens) * AU
    lat = np.radians(rng.uniform(-40.0, 40.0, n_ens))
    lon = rng.uniform(0.0, 2.0 * math.pi, n_ens)
    stop_h = rng.uniform(hours_lo, hours_hi, n_ens)
    ens = [Ensemble(n=int(counts[i]), ensemble=i, seed=seed, ekin=float(ekin[i]), r0=float(r0[i]),
                    lat0=float(lat[i]), lon0=float(lon[i]), lambda_par=float(lam[i]),
                    r_in=0.15 * AU, r_out=r_out_default(grid),
                    max_steps=int(round(stop_h[i] * HOUR / dt)))
           for i in range(n_ens)]
    return Workload(f"batched-{n_ens}ens-{total}", grid,
                    lambda g, device=None: fields.perturbed_parker(g, field_seed, device=device),
                    ens, dt, int(round(hours_hi * HOUR / dt)), store_dtype, 64)


def config_affine(n: int = 64, seed: int = 3) -> Workload:
    """Smooth right-hand side on a grid: affine field, no scattering, spread in
    radius and latitude; used for order-of-accuracy checks."""
    grid = SphericalGrid(32, 32, 16, 0.1 * AU, 2.0 * AU)
    ens = Ensemble(n=n, ensemble=0, seed=seed, r0=0.4 * AU, lat0=math.radians(10.0), dlat=math.radians(5.0),
                   dr0=0.05 * AU, lon0=1.0, dlon=0.5, lambda_par=0.0, r_in=0.15 * AU,
                   r_out=r_out_default(grid), mu_lo=-1.0, mu_hi=1.0)
    return Workload("affine-32x32x16", grid, lambda g, device=None: fields.affine(g), [ens], 1.0, 200, "f64", 0)
