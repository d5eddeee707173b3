"""Pins of the BF16 arithmetic model (bf16_model.py) from which the network
parity tolerances are derived: its rounding is round-to-nearest-even to 8
significant bits (unit roundoff 2^-8), and without rounding it is the
oracle's network exactly."""
import math

import numpy as np

import bf16_model as BM
from oracle import mlp_oracle as M
from synthetic import AU, SphericalGrid, fields


def test_bf16_rounding():
    rng = np.random.default_rng(0)
    x = rng.normal(size=100000) * 10.0 ** rng.uniform(-20, 20, size=100000)
    y = BM.bf16(x)
    assert np.all(np.abs(y - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))   # float32 step included
    assert np.max(np.abs(y - x) / np.abs(x)) > 0.9 * 2.0 ** -8          # and the bound is reached
    assert np.array_equal(BM.bf16(y), y)                                 # idempotent
    # ties go to the even significand: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert BM.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert BM.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def _net():
    """The network of the GPU parity tests (outputs biased away from zero)."""
    grid = SphericalGrid(24, 12, 16, 0.1 * AU, 2.0 * AU)
    f = fields.parker(grid)
    spec = M.make_spec(grid, f, seed=1)
    params = M.init_params(seed=2)
    params["Wo"] = 0.3 * params["Wo"]
    params["co"] = np.array([1.0, 0.3, -0.6, 0.2, 0.8, -0.4])
    return spec, {k: BM.bf16(v) for k, v in params.items()}


def test_without_rounding_the_model_is_the_oracle():
    spec, params = _net()
    rng = np.random.default_rng(1)
    n = 64
    pts = np.stack([rng.uniform(0.2, 1.8, n) * AU, rng.uniform(0.4, 2.7, n), rng.uniform(0, 6, n)])
    ident = lambda a: a
    ex = M.field(spec, params, *pts)
    mo = BM.field(spec, params, *pts, rnd=ident)
    assert np.allclose(mo, ex, rtol=1e-12, atol=1e-12 * np.abs(ex).max())
    p1, p2 = pts.T, pts.T + 1e-3 * rng.normal(size=(n, 3)) * np.array([AU, 1, 1])
    t1, t2 = rng.normal(size=(n, 6)), rng.normal(size=(n, 6))
    wc = np.ones(6)
    L, g = M.loss_and_grad(spec, params, p1, t1, p2, t2, wc, 2.0)
    Lm, gm = BM.loss_and_grad(spec, params, p1, t1, p2, t2, wc, 2.0, rnd=ident)
    assert Lm == L
    for k in g:
        assert np.array_equal(gm[k], g[k]), k


def test_rounded_network_errs_at_the_bf16_scale():
    """The model's output errors are a fraction of one BF16 rounding (2^-8):
    the outputs are sums over 128 rounded terms of both signs."""
    spec, params = _net()
    rng = np.random.default_rng(2)
    n = 512
    pts = np.stack([rng.uniform(0.2, 1.8, n) * AU, rng.uniform(0.4, 2.7, n), rng.uniform(0, 6, n)])
    ex = M.field(spec, params, *pts)
    errs = BM.field_errors(BM.field(spec, params, *pts), ex, BM.field_scales(spec, params, pts, ex))
    rms = math.sqrt(np.mean(errs["B"] ** 2))
    assert 2.0 ** -8 / 1000 < rms < 2.0 ** -8
