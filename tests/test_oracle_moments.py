"""Worked example for the oracle's snapshot moments (the statistics of Sect. 3:
<sin^2 alpha>(r), energy versus age near 1 AU, pitch-cosine distributions of
particles with at least one collision)."""
import math

import numpy as np

import oracle as O
from synthetic import AU, SphericalGrid, fields, C_LIGHT, M_ELECTRON, E_CHARGE
from synthetic.workloads import Ensemble

G = SphericalGrid(16, 8, 8, 0.1 * AU, 2.0 * AU)
BMAG = 1e-8


def _state(r, mu, status, k=0, step=0, t=0.0, ekin_ev=81000.0):
    m = M_ELECTRON
    gam = 1.0 + ekin_ev * E_CHARGE / (m * C_LIGHT ** 2)
    p = m * C_LIGHT * math.sqrt(gam * gam - 1.0)
    rec = np.zeros(1, dtype=O.PARTICLE_DTYPE)
    rec["r"], rec["th"], rec["ph"] = r, 1.5, 0.2
    rec["u"] = mu * p / m
    rec["mu_B"] = p * p * (1 - mu * mu) / (2 * m * BMAG)
    rec["status"], rec["k"], rec["step"], rec["t"] = status, k, step, t
    return rec


def test_worked_example():
    field = O.Field(G, fields.straight(G, BMAG))
    tab = O.make_ens_table([Ensemble(n=4, ensemble=0, seed=0)])
    parts = np.concatenate([
        _state(1.0 * AU, 0.6, O.ACTIVE, k=2, step=300, t=300.0),        # A
        _state(1.2 * AU, 0.1, O.EXITED, k=0, step=50, t=50.0),          # B
        _state(0.7 * AU, 0.3, O.FINISHED, k=5, step=100, t=100.0),      # C
        _state(0.55 * AU, -1.0, O.ACTIVE, k=0, step=5000, t=5000.0),    # D
    ])
    spec = O.MomentSpec(n_rbins=4, r_lo=0.0, r_hi=2.0 * AU, n_mubins=8,
                        sel_r_lo=0.5 * AU, sel_r_hi=1.5 * AU, age_lo=0.0, age_hi=1000.0, min_collisions=1,
                        n_agebins=3, age_max=6000.0, n_ebins=2, e_lo=80500.0, e_hi=82500.0)
    out = O.moments(field, tab, parts, spec)
    assert len(out) == 8 + 12 + 8 + 6
    assert list(out[0:4]) == [2, 1, 1, 0]
    assert out[4] == 7 and out[5] == 300 + 50 + 100 + 5000
    assert abs(out[6] - (2 ** 32 + math.floor(0.55 * 2 ** 32))) <= 2
    assert out[7] == 1
    rb = out[8:20].reshape(4, 3)
    assert list(rb[:, 0]) == [0, 1, 1, 0]
    assert abs(rb[2, 1] - math.floor(0.64 * 2 ** 32)) <= 1 and rb[1, 1] == 0
    assert abs(rb[2, 2] - 81000 * 65536) <= 1 and abs(rb[1, 2] - 81000 * 65536) <= 1
    mh = out[20:28]
    assert list(mh) == [0, 0, 0, 0, 0, 0, 1, 0]          # mu = 0.6 -> bin floor(1.6/2 * 8) = 6
    eh = out[28:34].reshape(3, 2)
    assert eh.tolist() == [[1, 0], [0, 0], [1, 0]]        # A: age 300 s, D: age 5000 s; both 81 keV
