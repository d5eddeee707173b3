"""Pins of the neural-field oracle: forward-mode tangents, the hand-written
gradient of the training loss, and grad|B|, (b.grad)b from the network's
derivatives, each against finite differences of the network itself."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M
from synthetic import AU, SphericalGrid, fields

GRID = SphericalGrid(16, 12, 16, 0.1 * AU, 2.0 * AU)


@pytest.fixture(scope="module")
def setup():
    data = fields.parker(GRID)
    spec = M.make_spec(GRID, data, seed=1)
    params = M.init_params(seed=2)
    rng = np.random.default_rng(3)
    n = 12
    pts = np.stack([rng.uniform(0.3, 1.8, n) * AU, rng.uniform(0.6, 2.5, n), rng.uniform(-3, 9, n)], axis=1)
    return spec, params, pts


def test_tangents_match_finite_differences(setup):
    spec, params, pts = setup
    h0, dh0 = M.features(spec, pts[:, 0], pts[:, 1], pts[:, 2])
    y, dy = M.forward_jvp(params, h0, dh0)
    steps = [1e-6 * AU, 1e-6, 1e-6]
    for d in range(3):
        e = np.zeros(3)
        e[d] = steps[d]
        hp, _ = M.features(spec, *(pts + e).T)
        hm, _ = M.features(spec, *(pts - e).T)
        fd = (M.forward(params, hp) - M.forward(params, hm)) / (2 * steps[d])
        assert np.allclose(dy[d], fd, rtol=1e-5, atol=1e-7 * np.abs(dy[d]).max())
    assert np.allclose(y, M.forward(params, h0))


def test_periodic_in_phi(setup):
    spec, params, pts = setup
    a = M.field(spec, params, pts[:, 0], pts[:, 1], pts[:, 2])
    b = M.field(spec, params, pts[:, 0], pts[:, 1], pts[:, 2] + 2 * math.pi)
    assert np.allclose(a, b, rtol=1e-9, atol=1e-30)


def test_loss_gradient_matches_finite_differences(setup):
    spec, params, pts = setup
    rng = np.random.default_rng(5)
    pts2 = pts + np.stack([rng.normal(0, 0.01 * AU, len(pts)), rng.normal(0, 0.01, len(pts)),
                           rng.normal(0, 0.01, len(pts))], axis=1)
    tgt = rng.normal(0, 1, (len(pts), 6)) * spec.scale
    tgt2 = tgt * 1.01
    wc = np.array([1.0, 0.5, 1.0, 2.0, 1.0, 0.5])
    L, g = M.loss_and_grad(spec, params, pts, tgt, pts2, tgt2, wc, beta=4.0)
    for name, idx in [("W1", (3, 7)), ("W4", (100, 2)), ("W6", (0, 127)), ("Wo", (2, 64)), ("c3", (11,)),
                      ("co", (4,)), ("c6", (90,))]:
        h = 1e-6
        p2 = {k: v.copy() for k, v in params.items()}
        p2[name][idx] += h
        Lp, _ = M.loss_and_grad(spec, p2, pts, tgt, pts2, tgt2, wc, 4.0)
        p2[name][idx] -= 2 * h
        Lm, _ = M.loss_and_grad(spec, p2, pts, tgt, pts2, tgt2, wc, 4.0)
        fd = (Lp - Lm) / (2 * h)
        assert g[name][idx] == pytest.approx(fd, rel=1e-4, abs=1e-9 * abs(L)), name


def _cart_basis(th, ph):
    st, ct, sp, cp = math.sin(th), math.cos(th), math.sin(ph), math.cos(ph)
    return (np.array([st * cp, st * sp, ct]), np.array([ct * cp, ct * sp, -st]), np.array([-sp, cp, 0.0]))


def test_gradB_and_curvature_from_network_derivatives(setup):
    """grad|B| and (b.grad)b of the neural field equal finite differences of
    its own B: checks the metric factors and connection terms."""
    spec, params, pts = setup

    def Bcart(x):
        r = np.linalg.norm(x)
        th = math.acos(x[2] / r)
        ph = math.atan2(x[1], x[0])
        v = M.field(spec, params, np.array([r]), np.array([th]), np.array([ph]))[0, 0:3]
        e = _cart_basis(th, ph)
        return v[0] * e[0] + v[1] * e[1] + v[2] * e[2]

    for i in range(6):
        r, th, ph = pts[i]
        f = M.field(spec, params, pts[i:i + 1, 0], pts[i:i + 1, 1], pts[i:i + 1, 2])[0]
        er, et, ep = _cart_basis(th, ph)
        x0 = r * er
        h = 1e-6 * r
        grad = np.zeros(3)
        for j, e in enumerate((er, et, ep)):
            grad[j] = (np.linalg.norm(Bcart(x0 + h * e)) - np.linalg.norm(Bcart(x0 - h * e))) / (2 * h)
        assert np.allclose(f[6:9], grad, rtol=1e-5, atol=1e-6 * np.abs(f[6:9]).max())
        b0 = Bcart(x0) / np.linalg.norm(Bcart(x0))
        bp = Bcart(x0 + h * b0); bp /= np.linalg.norm(bp)
        bm = Bcart(x0 - h * b0); bm /= np.linalg.norm(bm)
        Kc = (bp - bm) / (2 * h)
        K = np.array([Kc @ er, Kc @ et, Kc @ ep])
        assert np.allclose(f[9:12], K, rtol=1e-5, atol=1e-6 * np.abs(f[9:12]).max())


def test_callback_field_reproduces_builtin_field():
    """The callback field source (used to drive the oracle with the neural
    field) is plumbing only: fed the closed-form spiral it reproduces the
    built-in closed-form runs bit for bit, scattering included."""
    import oracle as O
    from dataclasses import replace
    from synthetic import B0_1AU, OMEGA_SUN, V_WIND
    from synthetic.workloads import Ensemble
    a0 = B0_1AU * AU * AU
    parker = {"a0": a0, "omega": OMEGA_SUN, "v_wind": V_WIND}
    grid = SphericalGrid(64, 32, 64, 0.1 * AU, 2.0 * AU)
    builtin = O.Field(grid, parker=parker)
    cb = O.Field(grid, callback=lambda r, th, ph: O.parker_closed_form(a0, OMEGA_SUN, V_WIND, r, th))
    ens = Ensemble(n=6, ensemble=0, seed=3, lambda_par=0.02 * AU, r_in=0.12 * AU, r_out=1.9 * AU)
    ens = replace(ens, r0=0.28 * AU, lat0=math.radians(24.0), lon0=0.1)
    tab = O.make_ens_table([ens])
    ids = np.arange(6, dtype=np.uint32)
    p1 = O.inject(builtin, tab, 0, ids)
    p2 = O.inject(cb, tab, 0, ids)
    assert p1.tobytes() == p2.tobytes()
    O.advance(builtin, tab, p1, 1.0, 400)
    O.advance(cb, tab, p2, 1.0, 400)
    assert p1["k"].sum() > 0                  # collisions happened
    assert p1.tobytes() == p2.tobytes()
