"""Pins of the full guiding-centre equations (Eqs. 1-2 with the terms that
carry derivatives of b and v_E) in the oracle, and of the node values of those
derivatives that the field builder provides.

* The builder's (v_E.grad)b, (b.grad)v_E and (v_E.grad)v_E (forward-mode
  automatic differentiation) equal central finite differences of b and v_E.
* Energy: for any field values, the right-hand side satisfies
    m c^2 dgamma/dt = q E.dR/dt + (mu_B/gamma) v_d.grad B
                      - gamma m (c_E |v_E|^2 + v_par v_E.(b.grad)v_E + v_E.(v_E.grad)v_E),
  with v_d the drift of the bracket and c_E = q v_par E_par / (gamma m c^2),
  an identity of Eqs. 1-2 (the (v_E.grad)b and (b.grad)b terms cancel between
  dR/dt and du/dt); a dropped, mis-signed or misplaced term breaks it.
* The drift terms the reduced form drops are of relative size u_sw / v (about
  3e-3 for 81 keV electrons in a 400 km/s wind) against the bracket's drifts it
  keeps (gradient, curvature, polarization).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from synthetic import AU, C_LIGHT, E_CHARGE, M_ELECTRON, SphericalGrid, V_WIND, fields
from synthetic.workloads import Ensemble

GRID = SphericalGrid(24, 16, 16, 0.2 * AU, 2.0 * AU)


def _b_vE(pos):
    """b and v_E = E x B / B^2 of the Parker spiral with E = -V r^ x B, plain evaluation."""
    B = torch.stack(fields.parker_B(pos[0], pos[1], pos[2]))
    rhat = pos / torch.sqrt((pos * pos).sum(0))
    E = -V_WIND * torch.linalg.cross(rhat, B, dim=0)
    B2 = (B * B).sum(0)
    return B / torch.sqrt(B2), torch.linalg.cross(E, B, dim=0) / B2


def test_builder_derivatives_match_finite_differences():
    extra = fields.parker_extra(GRID)
    rng = np.random.default_rng(4)
    checked = 0
    for _ in range(40):
        i, j, k = rng.integers(1, GRID.nr - 1), rng.integers(2, GRID.nth - 2), rng.integers(0, GRID.nph)
        r, th, ph = GRID.r_nodes()[i], GRID.th_nodes()[j], GRID.ph_nodes()[k]
        st, ct, sp, cp = math.sin(th), math.cos(th), math.sin(ph), math.cos(ph)
        x0 = torch.tensor([[r * st * cp], [r * st * sp], [r * ct]], dtype=torch.float64)
        b0, v0 = _b_vE(x0)
        h = 1e-4 * AU

        def ddir(fn_index, d):
            dn = d / torch.linalg.norm(d)
            fp = _b_vE(x0 + h * dn)[fn_index]
            fm = _b_vE(x0 - h * dn)[fn_index]
            return (fp - fm) / (2 * h) * torch.linalg.norm(d)

        A = ddir(0, v0)       # (v_E.grad) b
        Cv = ddir(1, b0)      # (b.grad) v_E
        D = ddir(1, v0)       # (v_E.grad) v_E
        basis = np.array([[st * cp, st * sp, ct], [ct * cp, ct * sp, -st], [-sp, cp, 0.0]])
        want = np.concatenate([basis @ v.numpy()[:, 0] for v in (A, Cv, D)])
        got = extra[i, j, k]
        for g in range(3):
            sl = slice(3 * g, 3 * g + 3)
            scale = np.linalg.norm(want[sl])
            assert np.linalg.norm(got[sl] - want[sl]) <= 1e-5 * scale + 1e-30, (g, got[sl], want[sl])
        checked += 1
    assert checked == 40


def _rand_state(rng):
    r = rng.uniform(0.3, 1.5) * AU
    th = rng.uniform(0.5, 2.6)
    u = rng.uniform(-1.5e8, 1.5e8)
    mu = rng.uniform(1e13, 1e16) * M_ELECTRON          # mu_B in J/T
    B = rng.normal(size=3) * 5e-9
    E = rng.normal(size=3) * 2e-3
    G = rng.normal(size=3) * 1e-19
    K = rng.normal(size=3) * 1e-11
    A = rng.normal(size=3) * 3e-6
    Cv = rng.normal(size=3) * 3e-6
    D = rng.normal(size=3) * 0.3
    return r, th, u, mu, np.concatenate([B, E, G, K]), np.concatenate([A, Cv, D])


@pytest.mark.parametrize("seed", range(6))
def test_energy_identity_of_full_equations(seed):
    rng = np.random.default_rng(100 + seed)
    q, m, c = -E_CHARGE, M_ELECTRON, C_LIGHT
    for _ in range(50):
        r, th, u, muB, fld, x = _rand_state(rng)
        F, vpar, gam = O.rhs([r, th, 0.3, u], muB, q, m, fld, extra=x)
        Rdot = np.array([F[0], r * F[1], r * math.sin(th) * F[2]])
        Bv, E, G = fld[0:3], fld[3:6], fld[6:9]
        Bm = np.linalg.norm(Bv)
        b = Bv / Bm
        vE = np.cross(E, b) / Bm
        Epar = E @ b
        A, Cv, D = x[0:3], x[3:6], x[6:9]
        mu = muB / m
        gdot = (u * F[3] + mu * (Rdot @ G)) / (gam * c * c)
        cE = q * vpar * Epar / (gam * m * c * c)
        v_d = Rdot - vpar * b - vE
        lhs = m * c * c * gdot
        rhs = q * (E @ Rdot) + (muB / gam) * (v_d @ G) - gam * m * (cE * (vE @ vE) + vpar * (Cv @ vE) + D @ vE)
        scale = abs(q * vpar * Epar) + abs(muB / gam * (Rdot @ G)) + gam * m * abs(vpar * (Cv @ vE))
        assert abs(lhs - rhs) <= 1e-10 * scale, (lhs, rhs)


def test_reduced_form_drops_terms_of_order_wind_over_speed():
    """Along electrons in the Parker spiral, the dR/dt and du/dt terms the
    reduced form drops are about u_sw / v of the drift terms it keeps."""
    f = fields.parker(GRID)
    x = fields.parker_extra(GRID)
    of = O.Field(GRID, f, extra=x)
    e = Ensemble(n=64, ensemble=0, seed=2, r0=0.6 * AU, lat0=math.radians(20.0), dlon=0.5, mu_lo=-1.0,
                 mu_hi=1.0, lambda_par=0.0, r_in=0.25 * AU, r_out=1.9 * AU)
    tab = O.make_ens_table([e])
    p = O.inject(of, tab, 0, np.arange(e.n, dtype=np.uint32))
    ratios = []
    for i in range(e.n):
        X = [p["r"][i], p["th"][i], p["ph"][i], p["u"][i]]
        g, ok = O.field_eval(of, *X[:3])
        xg, okx = O.field_eval_extra(of, *X[:3])
        assert ok and okx
        Ff, vpar, gam = O.rhs(X, p["mu_B"][i], e.q, e.m, g, extra=xg)
        Fr, _, _ = O.rhs(X, p["mu_B"][i], e.q, e.m, g)
        r, th = X[0], X[1]
        vec = lambda F: np.array([F[0], r * F[1], r * math.sin(th) * F[2]])
        Bm = np.linalg.norm(g[0:3])
        b = g[0:3] / Bm
        vE = np.cross(g[3:6], b) / Bm
        drift = np.linalg.norm(vec(Fr) - vpar * b - vE)      # the bracket's drifts of the reduced form
        dropped = np.linalg.norm(vec(Ff) - vec(Fr))
        ratios.append(dropped / drift)
    med = float(np.median(ratios))
    speed = C_LIGHT * math.sqrt(1 - (1 / (1 + 81e3 * E_CHARGE / (M_ELECTRON * C_LIGHT ** 2))) ** 2)
    assert 0.1 * V_WIND / speed < med < 10 * V_WIND / speed, (med, V_WIND / speed)


def test_full_equations_change_trajectories_slightly():
    """Integrated with and without the extra terms: the trajectories separate by
    far less than the drift displacement itself (the terms are small)."""
    f = fields.parker(GRID)
    x = fields.parker_extra(GRID)
    e = Ensemble(n=32, ensemble=0, seed=5, r0=0.5 * AU, lat0=math.radians(20.0), dlon=0.5, mu_lo=-1.0,
                 mu_hi=1.0, lambda_par=0.0, r_in=0.25 * AU, r_out=1.9 * AU)
    tab = O.make_ens_table([e])
    full = O.Field(GRID, f, extra=x)
    red = O.Field(GRID, f)
    p1 = O.inject(full, tab, 0, np.arange(e.n, dtype=np.uint32))
    p2 = p1.copy()
    O.advance(full, tab, p1, 1.0, 1200)
    O.advance(red, tab, p2, 1.0, 1200)
    act = (p1["status"] == O.ACTIVE) & (p2["status"] == O.ACTIVE)
    assert act.sum() > 10
    d = np.abs(p1["r"] - p2["r"])[act] / AU
    assert 0 < d.max() < 1e-3
