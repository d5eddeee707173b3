"""Pins of the oracle's guiding-centre right-hand side (Eqs. 1-2) against
textbook drifts, the paper's own drift formulas of Sect. 3, and the energy
identity that the reduced system satisfies."""
import math

import numpy as np
import pytest

import oracle as O
from synthetic import C_LIGHT, E_CHARGE, M_ELECTRON, AU

Q, M = -E_CHARGE, M_ELECTRON
C2 = C_LIGHT ** 2


def fld(B=(0, 0, 0), E=(0, 0, 0), G=(0, 0, 0), K=(0, 0, 0)):
    return np.array(list(B) + list(E) + list(G) + list(K), dtype=np.float64)


def gamma_of(u, mu_B, Bmag):
    return math.sqrt(1.0 + u * u / C2 + 2 * mu_B * Bmag / (M * C2))


R0, TH0 = 1.0 * AU, 1.2


def local_velocity(F, X):
    """(V_r, V_th, V_ph) from coordinate rates."""
    return np.array([F[0], X[0] * F[1], X[0] * math.sin(X[1]) * F[2]])


def test_straight_line_in_uniform_field():
    u = 1.3e8
    X = np.array([R0, TH0, 0.4, u])
    F, vpar, g = O.rhs(X, 0.0, Q, M, fld(B=(5e-9, 0, 0)))
    assert g == pytest.approx(math.sqrt(1 + u * u / C2), rel=1e-15)
    assert np.allclose(F, [u / g, 0, 0, 0], rtol=1e-15, atol=0)
    assert vpar == pytest.approx(u / g, rel=1e-15)


def test_exb_drift_sign_and_magnitude():
    # E = E0 th^, B = B0 ph^ : E x B / B^2 = (E0/B0) (th^ x ph^) = (E0/B0) r^
    E0, B0 = 2e-3, 6e-9
    X = np.array([R0, TH0, 0.0, 0.0])
    F, _, _ = O.rhs(X, 0.0, Q, M, fld(B=(0, 0, B0), E=(0, E0, 0)))
    assert np.allclose(local_velocity(F, X), [E0 / B0, 0, 0], rtol=1e-14, atol=1e-12)
    assert F[3] == 0.0


@pytest.mark.parametrize("charge", [Q, -Q])
def test_grad_b_drift_matches_paper_formula(charge):
    # paper Sect. 3: v_gradB = [gamma m v_perp^2 / (2 q B)] b x grad ln B
    B0, g = 6e-9, 3e-19
    mu_B = 2e-7
    X = np.array([R0, TH0, 0.0, 0.0])
    F, _, gam = O.rhs(X, mu_B, charge, M, fld(B=(B0, 0, 0), G=(0, g, 0)))
    vperp2 = 2 * mu_B * B0 / (M * gam * gam)               # mu_B = m gamma^2 v_perp^2 / (2B)
    want = gam * M * vperp2 / (2 * charge * B0) * np.cross([1, 0, 0], [0, g / B0, 0])
    assert np.allclose(local_velocity(F, X), want, rtol=1e-13, atol=1e-30)
    # b x grad B = g ph^ here, so the drift is along sign(q) ph^: opposite for opposite charges
    assert np.sign(local_velocity(F, X)[2]) == np.sign(charge)


def test_curvature_drift_matches_paper_formula():
    # paper Sect. 3: v_curv = [gamma m v_par^2 / (q B)] b x (b.grad) b
    B0, kap, u = 6e-9, 4e-12, 1.5e8
    X = np.array([R0, TH0, 0.0, u])
    F, vpar, gam = O.rhs(X, 0.0, Q, M, fld(B=(B0, 0, 0), K=(0, kap, 0)))
    want = np.array([vpar, 0, 0]) + gam * M * vpar ** 2 / (Q * B0) * np.cross([1, 0, 0], [0, kap, 0])
    assert np.allclose(local_velocity(F, X), want, rtol=1e-13)


def test_mirror_force_and_parallel_electric_field():
    B0, g, mu_B, u, Epar = 6e-9, 3e-19, 2e-7, 7e7, 1e-6
    X = np.array([R0, TH0, 0.0, u])
    F, _, gam = O.rhs(X, mu_B, Q, M, fld(B=(B0, 0, 0), E=(Epar, 0, 0), G=(g, 0, 0)))
    # d(gamma v_par)/dt = (q/m) E_par - mu_B/(gamma m) b.grad B  (Eq. 2)
    assert F[3] == pytest.approx(Q / M * Epar - mu_B / (gam * M) * g, rel=1e-14)


def test_drift_free_keeps_only_parallel_motion():
    rng = np.random.default_rng(0)
    f = fld(B=(5e-9, 1e-9, -3e-9), E=(0, 2e-3, 1e-4), G=(-2e-19, 1e-20, 0), K=(-2e-12, 1e-12, -3e-12))
    X = np.array([R0, TH0, 0.3, 9e7])
    F, vpar, _ = O.rhs(X, 1e-7, Q, M, f, drift_free=True)
    b = f[0:3] / np.linalg.norm(f[0:3])
    assert np.allclose(local_velocity(F, X), vpar * b, rtol=1e-14)
    del rng


@pytest.mark.parametrize("seed", range(8))
def test_energy_identity_of_reduced_system(seed):
    """With E.B = 0 the reduced Eqs. 1-2 give
        m c^2 d(gamma)/dt = q E.dR/dt + (mu_B/gamma) v_curv . grad|B|
    (paper Eq. 14 form q v_d.E plus the residual of the reduction), where
    d(gamma)/dt follows from gamma^2 = 1 + (u^2 + 2 mu_B B/m)/c^2 and dB/dt = dR/dt . grad|B|.
    A dropped or mis-signed term in Eq. 1 or Eq. 2 breaks the balance."""
    rng = np.random.default_rng(seed)
    B = rng.normal(size=3) * 5e-9
    wind = rng.normal(size=3) * 4e5
    E = -np.cross(wind, B)                     # ideal Ohm's law: E.B = 0
    G = rng.normal(size=3) * 3e-19
    K = rng.normal(size=3) * 3e-12
    mu_B = abs(rng.normal()) * 3e-7
    u = rng.normal() * 1e8
    X = np.array([rng.uniform(0.3, 1.8) * AU, rng.uniform(0.4, 2.7), rng.uniform(0, 6), u])
    f = fld(B, E, G, K)
    F, vpar, gam = O.rhs(X, mu_B, Q, M, f)
    Rdot = local_velocity(F, X)
    Bmag = np.linalg.norm(B)
    b = B / Bmag
    Bdot = Rdot @ G
    gdot = (u * F[3] + mu_B / M * Bdot) / (gam * C2)
    vc = gam * M * vpar ** 2 / (Q * Bmag) * np.cross(b, K)
    lhs = M * C2 * gdot
    rhs = Q * (E @ Rdot) + mu_B / gam * (vc @ G)
    # rounding scale: the parallel (mirror) exchange terms cancel inside lhs
    scale = (abs(Q * (E @ Rdot)) + abs(mu_B / gam * (vc @ G)) + abs(M * u * F[3] / gam)
             + abs(mu_B * Bdot / gam))
    assert abs(lhs - rhs) <= 1e-11 * scale
    # the balance is not trivially small: each side is a sizeable fraction of the scale
    assert abs(rhs) > 1e-6 * scale


def test_drift_free_rhs_conserves_energy():
    """Drift-free form with E_par = 0: no work along b and no drift across E, so gamma is constant."""
    rng = np.random.default_rng(11)
    B = rng.normal(size=3) * 5e-9
    E = -np.cross(rng.normal(size=3) * 4e5, B)
    G = rng.normal(size=3) * 3e-19
    K = rng.normal(size=3) * 3e-12
    mu_B, u = 2e-7, 1e8
    X = np.array([AU, 1.0, 0.0, u])
    F, vpar, gam = O.rhs(X, mu_B, Q, M, fld(B, E, G, K), drift_free=True)
    Rdot = local_velocity(F, X)
    gdot = (u * F[3] + mu_B / M * (Rdot @ G)) / (gam * C2)
    # drift-free: energy exactly conserved when E_par = 0 (no work along b, no drift across E)
    assert abs(M * C2 * gdot) <= 1e-12 * abs(M * u * F[3] / gam)
