"""The full guiding-centre equations (Eqs. 1-2 with the terms that carry
derivatives of b and v_E) on the device, through the C ABI, against the FP64
oracle.  The field carries a second node array with (v_E.grad)b, (b.grad)v_E
and (v_E.grad)v_E.

Bar (FP64 state): identical status, step count, collision count and collision
log for every electron; relative errors <= 1e-6 in position, u and mu_B after
2 h; the device's full-minus-reduced difference equals the oracle's."""
import numpy as np
import pytest

import paper_2403_06706_amd as gcp
from gpu_helpers import compare, field_of, generation, run_gpu, run_oracle, same_state, say, small, stored
from synthetic import AU, M_ELECTRON, fields

pytestmark = pytest.mark.gpu
TOL64 = 1e-6
_EXTRA = {}


def extra_of(wl):
    if wl.grid not in _EXTRA:
        _EXTRA[wl.grid] = fields.parker_extra(wl.grid)
    return _EXTRA[wl.grid]


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_full_equations_parity_fp64(store):
    wl = small()
    f = stored(field_of(wl), store)
    x = stored(extra_of(wl), store)
    say(f"full-equation parity, store={store}")
    st, log = run_gpu(wl, f, store_dtype=store, log_depth=64, extra=x)
    p, ologs, *_ = run_oracle(wl, f, log_depth=64, extra=x)
    pos, u, mu = compare(st, p, M_ELECTRON, TOL64, f"full store={store}")
    assert np.array_equal(log, ologs[0])
    say(f"  max rel err pos {pos.max():.2e} u {u.max():.2e} mu {mu.max():.2e}")
    assert p["k"].sum() > 1000


def test_full_minus_reduced_matches_oracle():
    wl = small(n=512, hours=0.25, lambda_par=0.0)        # no collisions: no decision can flip
    f = field_of(wl)
    x = extra_of(wl)
    sf, _ = run_gpu(wl, f, extra=x)
    sr, _ = run_gpu(wl, f)
    pf, *_ = run_oracle(wl, f, extra=x)
    pr, *_ = run_oracle(wl, f)
    act = (sf["status"] == 0) & (sr["status"] == 0) & (pf["status"] == 0) & (pr["status"] == 0)
    assert act.sum() > 100
    dd = (sf["r"] - sr["r"])[act]
    do = (pf["r"] - pr["r"])[act]
    say(f"  full - reduced in r after 15 min: max {np.abs(do).max() / AU:.3e} AU (oracle), "
        f"device - oracle {np.abs(dd - do).max() / AU:.3e} AU")
    assert np.abs(do).max() > 0
    assert np.abs(dd - do).max() <= 1e-9 * AU


def test_full_equations_forms_bitwise():
    """Throughput, all-pairs (the tail of the full equations), persistent grid and
    graph replay agree bit for bit, also with rebirth and wind-frame scattering."""
    wl = small(n=1024, hours=0.5, v_wind=418e3, r_out=0.7 * AU, rebirth_steps=10 ** 6)
    f = field_of(wl)
    x = extra_of(wl)
    ref, _ = run_gpu(wl, f, tail_threshold=0, extra=x)
    for kw in (dict(tail_threshold=2048), dict(tail_threshold=1 << 30), dict(persistent=True),
               dict(graph=True, chunk=60)):
        st, _ = run_gpu(wl, f, extra=x, **kw)
        same_state(ref, st)
    p, *_ = run_oracle(wl, f, extra=x)
    compare(ref, p, M_ELECTRON, TOL64, "full + wind + rebirth")
    assert np.array_equal(generation(ref), p["gen"]) and generation(ref).sum() > 500


def test_nonfinite_extra_array_marks_particles():
    """NaN in the extra node array over one radial shell: electrons that reach it
    end NONFINITE at the same step on both sides, a collision pending there
    applied first (the order of the field's own check), and the rest match."""
    from oracle import NONFINITE
    wl = small(n=600, hours=0.5, lambda_par=0.05 * AU)
    f = field_of(wl)
    x = extra_of(wl).copy()
    i = int((0.45 * AU - wl.grid.r_min) / wl.grid.dr)
    x[i, :, :, 7] = np.nan
    st, log = run_gpu(wl, f, log_depth=64, extra=x)
    p, ologs, *_ = run_oracle(wl, f, log_depth=64, extra=x)
    assert np.array_equal(st["status"], p["status"])
    assert np.array_equal(st["step"], p["step"]) and np.array_equal(st["k"], p["k"])
    assert np.array_equal(log, ologs[0])
    bad = p["status"] == NONFINITE
    assert bad.sum() > 10
    compare({k: v[~bad] for k, v in st.items()}, p[~bad], M_ELECTRON, TOL64, "finite part")


def test_full_equations_argument_errors():
    wl = small(n=4, hours=0.0)
    f = field_of(wl)
    ctx = gcp.Context(device=0)
    with pytest.raises(ValueError):
        ctx.load_field(wl.grid, f, "f64", extra=np.zeros((2, 2, 2, 9)))
    ctx.close()
    from oracle import mlp_oracle as M
    spec = M.make_spec(wl.grid, f, seed=1)
    ctx = gcp.Context(device=0, field_source="mlp")
    ctx.load_field(wl.grid, f, "f64", extra=extra_of(wl))
    ctx.mlp_set(spec.freq, spec.r_ref, spec.scale, spec.power, M.init_params(seed=2))
    ctx.inject(wl.ensembles[0])
    with pytest.raises(gcp.GCError, match="full"):
        ctx.advance(1.0, 1)
    ctx.close()
