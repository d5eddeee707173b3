"""Pins of the oracle's field evaluation (trilinear interpolation of the
gridded field, Sect. 2.2) and of its closed-form Parker spiral."""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle as O
from synthetic import AU, OMEGA_SUN, V_WIND, B0_1AU, SphericalGrid, fields

A0 = B0_1AU * AU * AU
PARKER = {"a0": A0, "omega": OMEGA_SUN, "v_wind": V_WIND}


def _cart_basis(th, ph):
    st, ct, sp, cp = math.sin(th), math.cos(th), math.sin(ph), math.cos(ph)
    return (np.array([st * cp, st * sp, ct]), np.array([ct * cp, ct * sp, -st]), np.array([-sp, cp, 0.0]))


def _closed(r, th):
    return O.parker_closed_form(A0, OMEGA_SUN, V_WIND, r, th)


def test_closed_form_matches_autodiff_grid_nodes():
    """Two independent derivations: hand-derived closed forms (oracle) and
    forward-mode autodiff of the Cartesian Parker field (input builder)."""
    g = SphericalGrid(12, 10, 8, 0.1 * AU, 2.0 * AU)
    data = fields.parker(g)
    for i in range(g.nr):
        for j in range(g.nth):
            want = _closed(g.r_nodes()[i], g.th_nodes()[j])
            for k in range(g.nph):
                got = data[i, j, k]
                for grp in range(4):
                    sl = slice(3 * grp, 3 * grp + 3)
                    scale = np.linalg.norm(want[sl]) + 1e-300
                    assert np.max(np.abs(got[sl] - want[sl])) <= 1e-12 * scale


@pytest.mark.parametrize("r_au,th", [(0.28, math.radians(66)), (1.0, math.radians(66)), (1.7, 1.2), (0.5, 2.2)])
def test_closed_form_gradients_vs_finite_differences(r_au, th):
    r = r_au * AU
    ph = 0.3
    f0 = _closed(r, th)

    def bmag(rr, tt):
        v = _closed(rr, tt)
        return np.linalg.norm(v[0:3])

    hr = 1e-5 * r
    ht = 1e-5
    G_fd = np.array([(bmag(r + hr, th) - bmag(r - hr, th)) / (2 * hr),
                     (bmag(r, th + ht) - bmag(r, th - ht)) / (2 * r * ht), 0.0])
    assert np.allclose(f0[6:9], G_fd, rtol=1e-7, atol=1e-9 * np.linalg.norm(f0[6:9]))

    # (b.grad) b: difference the Cartesian unit vector b along b itself
    def b_cart(x):
        rr = np.linalg.norm(x)
        tt = math.acos(x[2] / rr)
        pp = math.atan2(x[1], x[0])
        v = _closed(rr, tt)[0:3]
        e = _cart_basis(tt, pp)
        B = v[0] * e[0] + v[1] * e[1] + v[2] * e[2]
        return B / np.linalg.norm(B)

    er, et, ep = _cart_basis(th, ph)
    x0 = r * er
    b0 = b_cart(x0)
    h = 1e-5 * r
    K_cart = (b_cart(x0 + h * b0) - b_cart(x0 - h * b0)) / (2 * h)
    K_fd = np.array([K_cart @ er, K_cart @ et, K_cart @ ep])
    assert np.allclose(f0[9:12], K_fd, rtol=1e-6, atol=1e-8 * np.linalg.norm(f0[9:12]))
    # E = -V r^ x B for the radial wind (ideal Ohm's law, Sect. 2.2)
    Bv = f0[0:3]
    E_want = -V_WIND * np.cross([1.0, 0.0, 0.0], Bv)
    assert np.allclose(f0[3:6], E_want, rtol=1e-14, atol=1e-20)


def test_closed_form_curvature_tends_to_circle():
    """Far out (w -> inf) the spiral winds into circles about the axis: the
    curvature vector has magnitude 1/(r sin th) and points to the axis."""
    r, th = 2000 * AU, 1.0
    K = _closed(r, th)[9:12]
    rho = r * math.sin(th)
    want = -np.array([math.sin(th), math.cos(th), 0.0]) / rho   # -rho^ / rho in (r^, th^, ph^)
    assert np.allclose(K, want, rtol=1e-3, atol=1e-3 / rho)


def _random_grid(seed, nr=7, nth=6, nph=5):
    g = SphericalGrid(nr, nth, nph, 0.2 * AU, 1.5 * AU)
    rng = np.random.default_rng(seed)
    return g, rng.standard_normal(g.shape())


def test_trilinear_reproduces_nodes_and_matches_library_interpolator():
    g, data = _random_grid(0)
    F = O.Field(g, data)
    # nodes
    for (i, j, k) in [(0, 0, 0), (3, 2, 4), (g.nr - 1, g.nth - 1, g.nph - 1), (1, 5, 0)]:
        v, ok = O.field_eval(F, g.r_nodes()[i], g.th_nodes()[j], g.ph_nodes()[k])
        assert ok and np.allclose(v, data[i, j, k], rtol=1e-14, atol=1e-14)
    # brute force against scipy's RegularGridInterpolator on a phi-padded copy
    padded = np.concatenate([data, data[:, :, :1]], axis=2)
    ph_nodes = np.append(g.ph_nodes(), 2 * math.pi)
    interp = RegularGridInterpolator((g.r_nodes(), g.th_nodes(), ph_nodes), padded, method="linear")
    rng = np.random.default_rng(1)
    for _ in range(200):
        r = rng.uniform(g.r_min, g.r_max)
        th = rng.uniform(g.th_nodes()[0], g.th_nodes()[-1])
        ph = rng.uniform(0, 2 * math.pi)
        v, ok = O.field_eval(F, r, th, ph)
        assert ok
        assert np.allclose(v, interp([[r, th, ph]])[0], rtol=1e-12, atol=1e-12)


def test_trilinear_periodic_and_clamped():
    g, data = _random_grid(2)
    F = O.Field(g, data)
    r, th = 0.77 * AU, 1.3
    for ph in (0.1, 2.0, 6.2):
        a, _ = O.field_eval(F, r, th, ph)
        b, _ = O.field_eval(F, r, th, ph + 2 * math.pi)
        c, _ = O.field_eval(F, r, th, ph - 4 * math.pi)
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12) and np.allclose(a, c, rtol=1e-12, atol=1e-12)
    # outside the r range and theta node range the stencil clamps to the edge cell
    lo, _ = O.field_eval(F, 0.01 * AU, 0.01, 0.0)
    assert np.allclose(lo, data[0, 0, 0])
    hi, _ = O.field_eval(F, 9 * AU, math.pi - 0.01, 0.0)
    assert np.allclose(hi, data[-1, -1, 0])


def test_trilinear_is_exact_on_affine_field():
    g = SphericalGrid(9, 8, 6, 0.1 * AU, 2.0 * AU)
    data = fields.affine(g)
    F = O.Field(g, data)
    rng = np.random.default_rng(3)
    for _ in range(100):
        r = rng.uniform(g.r_min, g.r_max)
        th = rng.uniform(g.th_nodes()[0], g.th_nodes()[-1])
        ph = rng.uniform(-10, 10)
        v, ok = O.field_eval(F, r, th, ph)
        want = fields.affine_at(r, th)
        assert ok and np.allclose(v, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_nonfinite_inputs_and_nodes_are_flagged():
    g, data = _random_grid(4)
    F = O.Field(g, data)
    _, ok = O.field_eval(F, float("nan"), 1.0, 0.0)
    assert not ok
    _, ok = O.field_eval(F, 0.5 * AU, 1.0, float("inf"))
    assert not ok
    data2 = data.copy()
    data2[2, 2, 2, 5] = np.nan
    F2 = O.Field(g, data2)
    _, ok = O.field_eval(F2, g.r_nodes()[2], g.th_nodes()[2], g.ph_nodes()[2])
    assert not ok
