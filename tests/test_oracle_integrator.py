"""Pins of the oracle's time integration: the predictor-corrector of Eqs. 5-6
against Adams-type polynomial exactness and its error constant, observed third
order on a smooth field, and invariants that the setup fixes (field-line
invariant, energy, magnetic moment, mirror point)."""
import math
from dataclasses import replace

import numpy as np
import pytest

import oracle as O
from synthetic import AU, OMEGA_SUN, V_WIND, B0_1AU, C_LIGHT, E_CHARGE, M_ELECTRON, SphericalGrid, fields
from synthetic.workloads import Ensemble

A0 = B0_1AU * AU * AU
PARKER = {"a0": A0, "omega": OMEGA_SUN, "v_wind": V_WIND}
GRID = SphericalGrid(64, 32, 64, 0.1 * AU, 2.0 * AU)


# ---------------------------------------------------------------------------
# Eqs. 5-6 on dy/dt = f(t): a 1-D quadrature problem with known answer
# ---------------------------------------------------------------------------
def _step(f, tn, h, tau):
    hp = h / tau
    Fn, Fp, Fs = f(tn), f(tn - hp), f(tn + h)
    X = np.zeros(4)
    vec = lambda v: np.full(4, v)
    pred = O.pc_predict(X, vec(Fn), vec(Fp), h, tau)[0]
    corr = O.pc_correct(X, vec(Fn), vec(Fs), vec(Fp), h, tau)[0]
    return pred, corr


@pytest.mark.parametrize("tau", [0.5, 1.0, 2.0, 1.7])
def test_corrector_exact_for_quadratics_predictor_for_lines(tau):
    tn, h = 0.3, 0.25
    quad = lambda t: 2.0 - 3.0 * t + 5.0 * t * t
    line = lambda t: 1.5 + 4.0 * t
    exact_q = lambda a, b: (2.0 * b - 1.5 * b * b + 5.0 / 3.0 * b ** 3) - (2.0 * a - 1.5 * a * a + 5.0 / 3.0 * a ** 3)
    exact_l = lambda a, b: (1.5 * b + 2.0 * b * b) - (1.5 * a + 2.0 * a * a)
    _, corr = _step(quad, tn, h, tau)
    assert corr == pytest.approx(exact_q(tn, tn + h), rel=1e-13)
    pred, _ = _step(line, tn, h, tau)
    assert pred == pytest.approx(exact_l(tn, tn + h), rel=1e-13)
    # neither is exact one degree higher, so the scheme is not of higher order by accident
    cub = lambda t: t ** 3
    _, corr3 = _step(cub, tn, h, tau)
    assert abs(corr3 - ((tn + h) ** 4 - tn ** 4) / 4) > 1e-8
    pred2, _ = _step(quad, tn, h, tau)
    assert abs(pred2 - exact_q(tn, tn + h)) > 1e-8


def test_corrector_error_constant_at_constant_step():
    # 2-step Adams-Moulton: local error h^4 y''''/24; y' = t^3 about t_n = 0 gives h^4/4
    for h in (0.5, 0.1, 0.02):
        _, corr = _step(lambda t: t ** 3, 0.0, h, 1.0)
        assert corr - h ** 4 / 4 == pytest.approx(h ** 4 / 4, rel=1e-9)


# ---------------------------------------------------------------------------
# whole-particle runs on the closed-form Parker spiral
# ---------------------------------------------------------------------------
def _particle(field, ens, mu=0.5, r0=0.28 * AU, lat=math.radians(24.0), ph=0.1):
    e = replace(ens, r0=r0, lat0=lat, lon0=ph, dlon=0.0, dr0=0.0, dlat=0.0, mu_lo=mu, mu_hi=mu)
    tab = O.make_ens_table([e])
    p = O.inject(field, tab, 0, np.array([7], dtype=np.uint32))
    return p, tab


def _ens(**kw):
    base = dict(n=1, ensemble=0, seed=5, lambda_par=0.0, r_in=0.12 * AU, r_out=30 * AU)
    base.update(kw)
    return Ensemble(**base)


def test_third_order_convergence_on_smooth_field():
    field = O.Field(GRID, parker=PARKER)
    T = 512.0
    ens = _ens()
    finals = {}
    for dt in (0.125, 2.0, 4.0, 8.0, 16.0):
        p, tab = _particle(field, ens, mu=0.5)
        O.advance(field, tab, p, dt, int(round(T / dt)))
        assert p["status"][0] == O.ACTIVE
        finals[dt] = np.array([p["r"][0], p["th"][0], p["ph"][0], p["u"][0]])
    ref = finals[0.125]
    scale = np.array([AU, 1.0, 1.0, abs(ref[3])])
    err = {dt: np.max(np.abs(finals[dt] - ref) / scale) for dt in (2.0, 4.0, 8.0, 16.0)}
    orders = [math.log2(err[2 * dt] / err[dt]) for dt in (2.0, 4.0, 8.0)]
    assert all(2.6 < o < 3.4 for o in orders), (err, orders)


def test_field_line_invariant_drift_free_with_scattering():
    """Drift-free motion on the Parker spiral keeps th fixed and
    I = ph + (Omega/V) r constant; the scheme is linear in X with weights
    summing to one, so I is kept to round-off even across collisions."""
    field = O.Field(GRID, parker=PARKER)
    ens = _ens(drift_free=True, lambda_par=0.05 * AU, r_in=0.11 * AU, r_out=1.95 * AU)
    p, tab = _particle(field, ens, mu=0.7)
    th0 = p["th"][0]
    I0 = p["ph"][0] + OMEGA_SUN / V_WIND * p["r"][0]
    logs = O.advance(field, tab, p, 1.0, 3000, log_depth=8)
    assert p["k"][0] >= 3, "collisions expected"
    assert p["th"][0] == th0
    I1 = p["ph"][0] + OMEGA_SUN / V_WIND * p["r"][0]
    assert abs(I1 - I0) <= 1e-13 * abs(I0) + 1e-13
    del logs


def test_energy_invariant_without_magnetic_moment():
    """alpha = 0 injection (mu_B = 0) with all drifts, no scattering: with
    E = -grad Phi, Phi = -a0 Omega cos(th), W = (gamma-1) m c^2 + q Phi is
    conserved; the kinetic energy itself changes through the drift (Eq. 14)."""
    field = O.Field(GRID, parker=PARKER)
    ens = _ens()
    p, tab = _particle(field, ens, mu=1.0)
    assert p["mu_B"][0] == 0.0
    m, q, c2 = M_ELECTRON, -E_CHARGE, C_LIGHT ** 2

    def W(pp):
        g = math.sqrt(1.0 + pp["u"][0] ** 2 / c2)
        return (g - 1.0) * m * c2 + q * (-A0 * OMEGA_SUN * math.cos(pp["th"][0])), (g - 1.0) * m * c2

    W0, K0 = W(p)
    O.advance(field, tab, p, 1.0, 7200)
    assert p["status"][0] == O.ACTIVE
    W1, K1 = W(p)
    assert abs(K1 - K0) > 100 * E_CHARGE          # > 100 eV of drift-induced change
    assert abs(W1 - W0) < 1e-4 * abs(K1 - K0)


def test_energy_change_equals_drift_work_integral():
    """With mu_B != 0: Delta(gamma m c^2) = integral of [q E.dR/dt + (mu_B/gamma) v_curv.grad|B|] dt
    along the recorded trajectory (Simpson's rule over the 1 s steps)."""
    field = O.Field(GRID, parker=PARKER)
    ens = _ens()
    p, tab = _particle(field, ens, mu=0.4)
    mu_B = p["mu_B"][0]
    m, q, c2 = M_ELECTRON, -E_CHARGE, C_LIGHT ** 2
    n = 3600
    traj = O.advance_traj(field, tab, p, 1.0, n)
    assert p["status"][0] == O.ACTIVE
    P = np.zeros(n + 1)
    eng = np.zeros(n + 1)
    for i in range(n + 1):
        X = traj[i]
        f, ok = O.field_eval(field, X[0], X[1], X[2])
        F, vpar, g = O.rhs(X, mu_B, q, m, f)
        Rdot = np.array([F[0], X[0] * F[1], X[0] * math.sin(X[1]) * F[2]])
        Bmag = np.linalg.norm(f[0:3])
        vc = g * m * vpar ** 2 / (q * Bmag) * np.cross(f[0:3] / Bmag, f[9:12])
        P[i] = q * (f[3:6] @ Rdot) + mu_B / g * (vc @ f[6:9])
        eng[i] = g * m * c2
    integral = (P[0] + P[-1] + 4 * P[1:-1:2].sum() + 2 * P[2:-1:2].sum()) / 3.0
    dE = eng[-1] - eng[0]
    assert abs(dE) > 10 * E_CHARGE
    assert abs(dE - integral) < 1e-4 * abs(dE)


def test_magnetic_moment_constant_between_collisions():
    field = O.Field(GRID, parker=PARKER)
    p, tab = _particle(field, _ens(), mu=0.3)
    mu0 = p["mu_B"][0]
    O.advance(field, tab, p, 1.0, 2000)
    assert p["mu_B"][0] == mu0                     # Eq. 3, bitwise


def test_mirror_point_in_growing_field():
    """Radial B growing linearly with r: an electron moving outward with pitch
    cosine 1/2 mirrors where B = B(r0)/(1 - 1/4) (mu_B and |p| conserved)."""
    g = SphericalGrid(40, 16, 8, 0.1 * AU, 2.0 * AU)
    b1, ra, L = 1e-8, 0.3 * AU, 0.5 * AU
    field = O.Field(g, fields.mirror(g, b1, ra, L))
    ens = _ens(r_in=0.11 * AU, r_out=1.9 * AU)
    r0 = 0.3 * AU
    p, tab = _particle(field, ens, mu=0.5, r0=r0, lat=0.0)
    B0 = b1 * (1 + (r0 - ra) / L)
    r_m = ra + L * (B0 / 0.75 / b1 - 1)
    traj = O.advance_traj(field, tab, p, 0.5, 2400)
    rmax = np.nanmax(traj[:, 0])
    assert rmax == pytest.approx(r_m, rel=2e-6)
    assert traj[-1, 3] < 0                          # reflected
    u0 = traj[0, 3]
    gam = math.sqrt(1 + (u0 / 0.5) ** 2 / C_LIGHT ** 2)  # |p|/m = u0 / mu at injection
    del gam


def test_status_exit_finish_nonfinite():
    field = O.Field(GRID, parker=PARKER)
    # injected outside the shell -> EXITED at injection
    p, tab = _particle(field, _ens(r_in=0.3 * AU), mu=0.5, r0=0.28 * AU)
    assert p["status"][0] == O.EXITED
    # max_steps -> FINISHED exactly at that step
    p, tab = _particle(field, _ens(max_steps=37), mu=0.5)
    O.advance(field, tab, p, 1.0, 100)
    assert p["status"][0] == O.FINISHED and p["step"][0] == 37 and p["t"][0] == 37.0
    # outward exit -> EXITED with the step count at exit
    p, tab = _particle(field, _ens(r_out=0.3 * AU), mu=1.0)
    O.advance(field, tab, p, 1.0, 100)
    assert p["status"][0] == O.EXITED and p["r"][0] > 0.3 * AU and 0 < p["step"][0] < 100
    # a non-finite node value reached by the stencil -> NONFINITE
    g = SphericalGrid(16, 8, 8, 0.1 * AU, 2.0 * AU)
    data = fields.straight(g)
    data[5, :, :, 3] = np.nan
    fieldg = O.Field(g, data)
    p, tab = _particle(fieldg, _ens(r_in=0.11 * AU, r_out=1.8 * AU), mu=1.0, r0=0.3 * AU, lat=0.0)
    O.advance(fieldg, tab, p, 1.0, 2000)
    assert p["status"][0] == O.NONFINITE
