"""Pin of the E_par v_E term of the guiding-centre velocity (Eq. 1, Sect. 2.2).

As printed, the term (v_par/gamma) E_par v_E of Eq. 1 lacks a dimensional
factor; both sides read it as (q v_par E_par / (gamma m c^2)) v_E inside the
drift bracket.  In uniform fields (no gradient, no curvature) that term is the
only part of dR/dt that leaves the plane spanned by b and v_E: multiplied by
gamma m / (q B) it gives (v_par E_par / (B c^2)) b x v_E, a velocity along
E_perp.  Special relativity fixes it independently:

* In the frame S' moving with v_E, the transverse electric field vanishes and
  B' is tilted toward E_perp by E_par |E_perp| / (B^2 c^2).  A guiding centre
  moving along b' in S' moves, in the lab, with v_E plus a velocity whose
  components along E_perp and b stand in that ratio.
* A full-orbit (Boris) integration of the Lorentz force in the same fields
  drifts along E_perp by that fraction of its displacement along b.

A flipped sign, a dropped or extra q/(m c^2), or a wrong power of gamma in the
oracle's coefficient fails both checks (the first one for every charge, state
and pitch)."""
import math

import numpy as np
import pytest

import oracle as O
from synthetic import C_LIGHT, E_CHARGE, M_ELECTRON, AU

C = C_LIGHT


def lorentz_boost(beta):
    """4x4 boost to a frame moving with velocity beta c (contravariant components)."""
    b2 = float(beta @ beta)
    g = 1.0 / math.sqrt(1.0 - b2)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = -g * beta
    L[1:, 1:] += (g - 1.0) * np.outer(beta, beta) / b2
    return L


def field_tensor(E, B):
    """F^{mu nu}: F^{i0} = E_i / c, F^{ij} = -eps_ijk B_k."""
    F = np.zeros((4, 4))
    F[1:, 0] = E / C
    F[0, 1:] = -E / C
    F[1, 2], F[1, 3], F[2, 3] = -B[2], B[1], -B[0]
    F[2, 1], F[3, 1], F[3, 2] = B[2], -B[1], B[0]
    return F


def fields_from_tensor(F):
    E = C * F[1:, 0]
    B = np.array([F[3, 2], F[1, 3], F[2, 1]])
    return E, B


def setup(seed, e_par_over_cB=1e-2, vE_over_c=1e-3, B0=5e-9):
    """Uniform fields in the local spherical basis: |B| = B0 along a random
    direction, E = E_par b + E_perp with |E_perp| = vE B0."""
    rng = np.random.default_rng(seed)
    b = rng.normal(size=3)
    b /= np.linalg.norm(b)
    p = rng.normal(size=3)
    p -= (p @ b) * b
    e_perp = p / np.linalg.norm(p)
    E = e_par_over_cB * C * B0 * b + vE_over_c * C * B0 * e_perp
    return b * B0, E, b, e_perp


def oracle_ratio(B, E, b, e_perp, u, mu_B, q):
    """(V . e_perp) / (V . b) of the oracle's dR/dt at one point."""
    r, th = 1.0 * AU, 1.1
    fld = np.concatenate([B, E, np.zeros(6)])
    F, vpar, _ = O.rhs(np.array([r, th, 0.3, u]), mu_B, q, M_ELECTRON, fld)
    V = np.array([F[0], r * F[1], r * math.sin(th) * F[2]])
    assert V @ b == pytest.approx(vpar, rel=1e-12)      # uniform field: V.b = v_par exactly
    return (V @ e_perp) / (V @ b)


def boosted_ratio(B, E, b, e_perp, w=0.5 * C):
    """The same ratio from special relativity: boost the fields to the frame
    moving with v_E, move along b' there, and boost the velocity back."""
    vE = np.cross(E, B) / (B @ B)
    L = lorentz_boost(vE / C)
    Ep, Bp = fields_from_tensor(L @ field_tensor(E, B) @ L.T)
    # checks of the boost itself: field invariants, and no E' across b in S'
    assert Ep @ Bp == pytest.approx(E @ B, rel=1e-12)
    assert Bp @ Bp - Ep @ Ep / C**2 == pytest.approx(B @ B - E @ E / C**2, rel=1e-12)
    assert np.linalg.norm(np.cross(Ep, b)) <= 1e-12 * np.linalg.norm(Ep)
    bp = Bp / np.linalg.norm(Bp)
    gw = 1.0 / math.sqrt(1.0 - (w / C) ** 2)
    U = lorentz_boost(-vE / C) @ np.concatenate([[gw * C], gw * w * bp])
    V = C * U[1:] / U[0]
    assert V @ np.cross(b, e_perp) == pytest.approx(vE @ np.cross(b, e_perp), rel=1e-9)   # E x B drift kept
    return (V @ e_perp) / (V @ b), float(bp @ e_perp)


@pytest.mark.parametrize("seed", range(6))
def test_coefficient_matches_lorentz_transformation(seed):
    B, E, b, e_perp = setup(seed)
    want, tilt = boosted_ratio(B, E, b, e_perp)
    # the tilt is the physical effect being pinned: E_par |E_perp| / (B c)^2 = 1e-5 here
    assert tilt == pytest.approx(1e-5, rel=1e-4)
    for q in (-E_CHARGE, E_CHARGE):
        for u in (1.7e8, -0.9e8, 4.0e8):
            for mu_B in (0.0, 3e-7):
                got = oracle_ratio(B, E, b, e_perp, u, mu_B, q)
                # the reduced equations neglect O(v_E^2 / c^2) = 1e-6 relative
                assert got == pytest.approx(want, rel=2e-5), (q, u, mu_B)


def test_ratio_does_not_depend_on_the_boosted_speed():
    B, E, b, e_perp = setup(7)
    r1, _ = boosted_ratio(B, E, b, e_perp, w=0.1 * C)
    r2, _ = boosted_ratio(B, E, b, e_perp, w=-0.9 * C)
    assert r1 == pytest.approx(r2, rel=1e-9)


def boris_displacement(B, E, q, m, u0, dt, n):
    """Relativistic Boris integration of du/dt = (q/m)(E + v x B), u = gamma v,
    from x = 0; returns x after n steps."""
    qm = q / m
    x = np.zeros(3)
    u = u0.copy()
    for _ in range(n):
        um = u + 0.5 * dt * qm * E
        g = math.sqrt(1.0 + (um @ um) / C**2)
        t = 0.5 * dt * qm * B / g
        up = um + np.cross(um, t)
        s = 2.0 * t / (1.0 + t @ t)
        u = um + np.cross(up, s) + 0.5 * dt * qm * E
        x += dt * u / math.sqrt(1.0 + (u @ u) / C**2)
    return x


@pytest.mark.parametrize("seed", [0, 1])
def test_coefficient_matches_full_orbit_integration(seed):
    """An electron at 81 keV accelerated along b by E_par over about 2.5e8 m
    (gamma 1.16 -> about 2), with v_E = 3e5 m/s: its displacement along E_perp
    is the oracle's ratio times its displacement along b (about 300 m
    against a gyration residue below 1 m)."""
    B0 = 5e-9
    B, E, b, e_perp = setup(seed, e_par_over_cB=2e-3 / (C * B0), vE_over_c=3e5 / C, B0=B0)
    q, m = -E_CHARGE, M_ELECTRON
    vE = np.cross(E, B) / (B @ B)
    gamma0 = 1.0 + 81e3 * E_CHARGE / (m * C**2)
    upar = -math.sqrt(gamma0**2 - 1.0) * C          # along -b: q E_par < 0 accelerates it
    vpar = upar / gamma0
    v0 = vE + vpar * b                              # start on the drift, no gyration to speak of
    u0 = v0 / math.sqrt(1.0 - (v0 @ v0) / C**2)
    omega = E_CHARGE * B0 / (gamma0 * m)
    dt = 0.05 / omega
    x = boris_displacement(B, E, q, m, u0, dt, n=int(1.0 / dt))
    got = (x @ e_perp) / (x @ b)
    want = oracle_ratio(B, E, b, e_perp, upar, 0.0, q)
    assert abs(x @ e_perp) > 100.0                  # a drift of some hundred metres ...
    assert got == pytest.approx(want, rel=1e-2)     # ... in the oracle's proportion
    # and not the proportion of a flipped sign or of an extra 1/gamma
    assert abs(got + want) > 1.9 * abs(want)
    assert abs(got - want / gamma0) > 0.1 * abs(want)
