"""Seeded set-up of the neural field: architecture constants, Fourier
frequencies, output normalization and initial weights.  These are inputs (a
choice of hyperparameters and a seeded initialization), not arithmetic of the
method; the oracle and the HIP library both take them as given.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict

import numpy as np

N_FREQ = 64      # Fourier frequencies (128 features: sin and cos)
WIDTH = 128      # hidden width
DEPTH = 6        # hidden layers
N_OUT = 6        # B (3) and E (3), normalized


@dataclass
class MLPSpec:
    r_min: float
    r_max: float
    r_ref: float
    scale: np.ndarray      # [6] S_c
    power: np.ndarray      # [6] p_c
    freq: np.ndarray       # [64, 3]: a_j, b_j, n_j


def init_params(seed: int = 0) -> Dict[str, np.ndarray]:
    rng = np.random.default_rng(seed)
    p = {}
    for l in range(1, DEPTH + 1):
        p[f"W{l}"] = rng.normal(0.0, math.sqrt(2.0 / WIDTH), (WIDTH, WIDTH))
        p[f"c{l}"] = np.zeros(WIDTH)
    p["Wo"] = rng.normal(0.0, math.sqrt(1.0 / WIDTH), (N_OUT, WIDTH))
    p["co"] = np.zeros(N_OUT)
    return p


def make_spec(grid, field_data, seed: int = 0, sigma: float = 3.0, n_max: int = 8) -> MLPSpec:
    """Frequencies and output normalization for a field on a grid: a_j, b_j ~
    N(0, sigma^2), n_j uniform integers in [-n_max, n_max]; S_c the rms of
    component c times (r/r_ref)^p_c over the grid, floored at 1e-3 of the
    largest such rms of its vector (B or E), so that a component that vanishes
    on the grid (B_th and E_r of the plain spiral) keeps a usable scale."""
    rng = np.random.default_rng(seed)
    freq = np.stack([rng.normal(0, sigma, N_FREQ), rng.normal(0, sigma, N_FREQ),
                     rng.integers(-n_max, n_max + 1, N_FREQ).astype(np.float64)], axis=1)
    power = np.array([2.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    r_ref = 0.5 * (grid.r_min + grid.r_max)
    r = grid.r_nodes()[:, None, None]
    scale = np.empty(6)
    for c in range(6):
        v = field_data[..., c] * (r / r_ref) ** power[c]
        scale[c] = float(np.sqrt(np.mean(v ** 2)))
    for g in (slice(0, 3), slice(3, 6)):
        top = max(scale[g].max(), 1e-300)
        scale[g] = np.maximum(scale[g], 1e-3 * top)
    return MLPSpec(grid.r_min, grid.r_max, r_ref, scale, power, freq)
