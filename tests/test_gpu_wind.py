"""Scattering in the frame of the solar wind (Sect. 3.3) on the device, through
the C ABI, against the FP64 oracle.

Bar (FP64 state): identical status, step count, collision count and collision
log for every electron; relative errors <= 1e-6 in position, u and mu_B after
2 h.  Cases: all drifts, and only v_par b kept (the setting of Fig. 11); the
inertial-frame law of Eq. 10 and the law of Eq. 12; with rebirth on."""
import numpy as np
import pytest

import oracle as O
import paper_2403_06706_amd as gcp
from gpu_helpers import compare, field_of, generation, run_gpu, run_oracle, same_state, say, small, stored
from synthetic import AU, M_ELECTRON

pytestmark = pytest.mark.gpu
TOL64 = 1e-6
U_SW = 418e3


@pytest.mark.parametrize("drift_free,law,store", [(True, 0, "f64"), (False, 0, "f32"), (False, 1, "f64")])
def test_wind_frame_parity_fp64(drift_free, law, store):
    wl = small(v_wind=U_SW, drift_free=drift_free, scatter_law=law)
    f = stored(field_of(wl), store)
    say(f"wind-frame parity drift_free={drift_free} law={law} store={store}")
    st, log = run_gpu(wl, f, store_dtype=store, log_depth=64)
    p, ologs, *_ = run_oracle(wl, f, log_depth=64)
    pos, u, mu = compare(st, p, M_ELECTRON, TOL64, f"wind drift_free={drift_free} law={law}")
    assert np.array_equal(log, ologs[0])
    say(f"  collisions {int(p['k'].sum())}, max rel err pos {pos.max():.2e} u {u.max():.2e} mu {mu.max():.2e}")
    assert p["k"].sum() > 1000


def test_wind_frame_cools_against_inertial_frame():
    """Same electrons, same draws: with the centres moving with the wind the
    mean kinetic energy after 2 h is lower than with centres at rest, on both
    sides, by the same amount."""
    base = small(n=2048, drift_free=True)
    wind = small(n=2048, drift_free=True, v_wind=U_SW)
    f = field_of(base)
    out = {}
    for name, wl in (("rest", base), ("wind", wind)):
        st, _ = run_gpu(wl, f)
        p, *_ = run_oracle(wl, f)
        act = (st["status"] == 0) & (p["status"] == 0)
        out[name] = (st, p, act)
    # p^2 from each side's own state and its own |B| sampling
    from gpu_helpers import device_bmag, oracle_bmag
    of = O.Field(base.grid, f)
    drop = {}
    for name in ("rest", "wind"):
        st, p, act = out[name]
        bd = device_bmag(base, f, "f64", st["r"][act], st["th"][act], st["ph"][act])
        bo = oracle_bmag(of, p["r"][act], p["th"][act], p["ph"][act])
        pd = st["u"][act] ** 2 + 2 * st["mu"][act] * bd
        po = p["u"][act] ** 2 + 2 * (p["mu_B"][act] / M_ELECTRON) * bo
        drop[name] = (pd.mean(), po.mean())
    rel_dev = drop["wind"][0] / drop["rest"][0] - 1
    rel_ora = drop["wind"][1] / drop["rest"][1] - 1
    say(f"  mean p^2 change from wind-frame scattering: device {rel_dev:.3e}, oracle {rel_ora:.3e}")
    assert rel_ora < -1e-3                                  # cooling
    assert abs(rel_dev - rel_ora) <= 1e-6


def test_wind_frame_forms_and_rebirth_bitwise():
    """Throughput, latency forms, persistent grid and graph replay agree bit for
    bit with wind-frame scattering and rebirth on."""
    wl = small(n=1024, hours=0.5, v_wind=U_SW, r_out=0.7 * AU, rebirth_steps=10 ** 6)
    f = field_of(wl)
    ref, _ = run_gpu(wl, f, tail_threshold=0)
    for kw in (dict(tail_threshold=2048), dict(tail_threshold=1 << 30), dict(persistent=True),
               dict(graph=True, chunk=60)):
        st, _ = run_gpu(wl, f, **kw)
        same_state(ref, st)
    p, *_ = run_oracle(wl, f)
    compare(ref, p, M_ELECTRON, TOL64, "wind + rebirth")
    assert np.array_equal(generation(ref), p["gen"]) and generation(ref).sum() > 500


def test_wind_argument_errors():
    wl = small(n=4, hours=0.0)
    f = field_of(wl)
    ctx = gcp.Context(device=0)
    ctx.load_field(wl.grid, f, "f64")
    for bad in (-1.0, 0.2 * 299792458.0, float("nan")):
        with pytest.raises(gcp.GCError):
            ctx.inject(small(n=4, v_wind=bad).ensembles[0])
    ctx.close()
    from oracle import mlp_oracle as M
    spec = M.make_spec(wl.grid, f, seed=1)
    ctx = gcp.Context(device=0, field_source="mlp")
    ctx.load_field(wl.grid, f, "f64")
    ctx.mlp_set(spec.freq, spec.r_ref, spec.scale, spec.power, M.init_params(seed=2))
    ctx.inject(small(n=4, v_wind=U_SW).ensembles[0])
    with pytest.raises(gcp.GCError, match="wind"):
        ctx.advance(1.0, 1)
    ctx.close()
