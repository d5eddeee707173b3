"""Trilinear sampling of the packed field on the device (gc_field_sample)
against the oracle's interpolation of the same stored values, for every
storage type, on grids whose sizes leave partial node blocks (nr not a
multiple of 4, nph + 1 odd or even), at points that cover the r and theta
edges (where the stencil is clamped), the phi wrap and negative phi.

The stored values are what the library keeps: the float64 input, its float32
rounding, or for FP16 the input times a per-component power of two (chosen
from the component's largest magnitude) rounded once to half.
The oracle reads those numbers, so the two sides differ only in the rounding
of the interpolation (bar: 1e-12 of the component's largest magnitude).
A wrong block, chunk or stride in the layout moves values between nodes or
components and fails by orders of magnitude."""
import math

import numpy as np
import pytest

import oracle as O
import paper_2403_06706_amd as gcp
from gpu_helpers import say
from synthetic import AU, SphericalGrid

pytestmark = pytest.mark.gpu

GRIDS = [SphericalGrid(61, 30, 37, 0.1 * AU, 2.0 * AU), SphericalGrid(62, 31, 36, 0.1 * AU, 2.0 * AU),
         SphericalGrid(64, 32, 64, 0.1 * AU, 2.0 * AU), SphericalGrid(2, 2, 2, 0.5 * AU, 1.5 * AU),
         SphericalGrid(5, 3, 3, 0.2 * AU, 1.0 * AU)]


def stored_values(f, store):
    """The numbers the device holds for each storage type, as float64."""
    if store == "f64":
        return f
    if store == "f32":
        return f.astype(np.float32).astype(np.float64)
    mx = np.abs(f).reshape(-1, 12).max(axis=0)
    e = np.ceil(np.log2(mx)) - 14
    h = (f * np.exp2(-e)).astype(np.float16)        # one rounding from double, to nearest even
    return h.astype(np.float64) * np.exp2(e)


def sample_points(g, n, rng):
    dr = (g.r_max - g.r_min) / (g.nr - 1)
    r = rng.uniform(g.r_min - 0.5 * dr, g.r_max + 0.5 * dr, n)
    th = rng.uniform(1e-3, math.pi - 1e-3, n)
    ph = rng.uniform(-4 * math.pi, 4 * math.pi, n)
    # exact nodes and cell faces too
    k = n // 8
    r[:k] = g.r_min + rng.integers(0, g.nr, k) * dr
    th[:k] = (rng.integers(0, g.nth, k) + 0.5) * math.pi / g.nth
    ph[:k] = rng.integers(-g.nph, 2 * g.nph, k) * 2 * math.pi / g.nph
    return r, th, ph


@pytest.mark.parametrize("store", ["f64", "f32", "f16"])
@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_device_sampling_matches_oracle(gi, store):
    import torch
    g = GRIDS[gi]
    rng = np.random.default_rng(10 + gi)
    f = rng.normal(size=(g.nr, g.nth, g.nph, 12)) * np.exp2(rng.integers(-40, 10, 12))
    ctx = gcp.Context(device=0)
    ctx.load_field(g, f, store)
    r, th, ph = sample_points(g, 4000, rng)
    pts = torch.tensor(np.stack([r, th, ph]), dtype=torch.float64, device="cuda:0").contiguous()
    got = ctx.field_sample(pts).cpu().numpy()
    ctx.close()
    of = O.Field(g, stored_values(f, store))
    want = np.array([O.field_eval(of, r[i], th[i], ph[i])[0] for i in range(len(r))])
    scale = np.abs(f).reshape(-1, 12).max(axis=0)
    err = (np.abs(got - want) / scale).max()
    say(f"  grid {g.nr}x{g.nth}x{g.nph} store {store}: max error / component scale {err:.2e}")
    assert err <= 1e-12


def test_packed_field_limit():
    """A field whose packed form would exceed 4 GiB is refused before any
    value is read (the gathers use 32-bit byte offsets)."""
    import ctypes as C
    from paper_2403_06706_amd import _abi
    ctx = gcp.Context(device=0)
    small = np.zeros(12)
    d = _abi.gc_field_desc(1024, 512, 512, _abi.GC_F64, 0.1 * AU, 2.0 * AU, small.ctypes.data, _abi.GC_F32, 0, None)
    assert gcp.lib.gc_load_field(ctx._h, C.byref(d)) == _abi.GC_EINVAL
    assert b"4 GiB" in gcp.lib.gc_last_error(ctx._h)
    with pytest.raises(ValueError):
        ctx.load_field(GRIDS[0], np.zeros((3, 3, 3, 12)), "f32")
    ctx.close()
