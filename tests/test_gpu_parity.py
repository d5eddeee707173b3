"""Per-particle parity of the HIP path with the FP64 oracle, through the C ABI.

Bar (FP64 arithmetic on the GPU): identical status, step count and collision
count for every particle, relative errors <= 1e-6 in position, u = gamma v_par
and mu_B after 2 h of 1 s steps (the bar for the FP64 form).
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import oracle as O
from gpu_helpers import field_of, stored, run_gpu, run_oracle, compare, small, say
from synthetic import AU, M_ELECTRON, SphericalGrid, fields
from synthetic.workloads import Workload, Ensemble

pytestmark = pytest.mark.gpu
TOL64 = 1e-6


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_small_config_parity_fp64(store):
    """1,024 electrons, Parker spiral on 64x32x64, lambda = 0.5 AU, 7,200 steps."""
    wl = small()
    f = stored(field_of(wl), store)
    say(f"parity small config, store={store}")
    st, log = run_gpu(wl, f, store_dtype=store, log_depth=64)
    p, ologs, *_ = run_oracle(wl, f, log_depth=64)
    pos, u, mu = compare(st, p, M_ELECTRON, TOL64, f"store={store}")
    say(f"  max rel err pos {pos.max():.2e} u {u.max():.2e} mu {mu.max():.2e}; "
        f"exited {np.sum(p['status'] == O.EXITED)}, collisions {p['k'].sum()}")
    assert p["k"].sum() > 1000 and np.sum(p["status"] == O.EXITED) > 100   # the run exercises both
    # collision logs (steps at which each collision was applied) identical
    assert np.array_equal(log, ologs[0])


@pytest.mark.parametrize("n", [1, 63, 65, 257, 3000])
def test_ragged_sizes(n):
    wl = small(n=n, hours=0.25)
    f = field_of(wl)
    say(f"parity ragged n={n}")
    st, _ = run_gpu(wl, f, chunk=37)
    p, *_ = run_oracle(wl, f)
    compare(st, p, M_ELECTRON, TOL64, f"n={n}")


def test_empty_context_and_zero_steps():
    wl = small(n=0, hours=0.1)
    f = field_of(wl)
    st, _ = run_gpu(wl, f)
    assert len(st["r"]) == 0
    wl2 = small(n=50, hours=0.0)
    st2, _ = run_gpu(wl2, f, n_steps=0)
    p, *_ = run_oracle(wl2, f, n_steps=0)
    assert np.array_equal(st2["r"], p["r"]) and np.array_equal(st2["th"], p["th"])
    assert np.allclose(st2["u"], p["u"], rtol=1e-15, atol=0)   # |p|/m rounded in a different order
    assert np.allclose(st2["mu"], p["mu_B"] / M_ELECTRON, rtol=1e-14)
    assert np.allclose(st2["ell"], p["ell"], rtol=1e-15, atol=0)   # log() of two libraries


def test_injection_outside_shell_and_finish():
    wl = small(n=300, hours=0.2, r_in=0.281 * AU, max_steps=500, dr0=0.01 * AU)
    f = field_of(wl)
    st, _ = run_gpu(wl, f)
    p, *_ = run_oracle(wl, f)
    compare(st, p, M_ELECTRON, TOL64, "exit/finish")
    assert np.sum(p["status"] == O.EXITED) > 10 and np.sum(p["status"] == O.FINISHED) > 10


def test_nonfinite_field_marks_particles():
    wl = small(n=400, hours=0.5)
    f = field_of(wl).copy()
    i = int((0.6 * AU - wl.grid.r_min) / wl.grid.dr)
    f[i, :, :, 4] = np.nan
    st, _ = run_gpu(wl, f)
    p, *_ = run_oracle(wl, f)
    assert np.array_equal(st["status"], p["status"])
    assert np.sum(p["status"] == O.NONFINITE) > 10
    ok = p["status"] != O.NONFINITE
    sub = {k: v[ok] for k, v in st.items()}
    compare(sub, p[ok], M_ELECTRON, TOL64, "finite part")
    assert np.array_equal(st["step"], p["step"]) and np.array_equal(st["k"], p["k"])


@pytest.mark.parametrize("store", ["f64", "f32"])
@pytest.mark.parametrize("tail", [0, 1000])
def test_untame_field_gives_the_same_bits(store, tail):
    """One node value above 1e30, far from every electron, makes the field
    not tame: the push then tests each gather's result for non-finite values
    (a tame field lets the throughput and all-pairs forms skip the test).
    Both give the same bits.  tail 0: the throughput form throughout; 1000:
    the all-pairs form, then the quad form below 250 electrons."""
    from gpu_helpers import same_state
    wl = small(n=500, hours=0.5)
    f = field_of(wl)
    g = f.copy()
    g[-1, 0, 0, 11] = 2e30        # outermost shell, first theta row: never gathered
    say(f"tame/untame field, store={store}, tail={tail}")
    a, _ = run_gpu(wl, f, store_dtype=store, tail_threshold=tail)
    b, _ = run_gpu(wl, g, store_dtype=store, tail_threshold=tail)
    same_state(a, b)
    assert np.sum(a["status"] == O.EXITED) > 10


def test_drift_free_and_flux_weighted_law():
    wl = small(n=500, hours=0.5, drift_free=True, scatter_law=1, lambda_par=0.05 * AU)
    f = field_of(wl)
    st, _ = run_gpu(wl, f)
    p, *_ = run_oracle(wl, f)
    compare(st, p, M_ELECTRON, TOL64, "drift-free")
    assert p["k"].sum() > 500


def test_several_ensembles_and_variable_step():
    wl = small(n=200, hours=0.2)
    e0 = wl.ensembles[0]
    ens = [replace(e0, ensemble=0, n=200),
           replace(e0, ensemble=1, n=150, seed=7, lambda_par=0.1 * AU, ekin=e0.ekin * 3, lat0=-0.3),
           replace(e0, ensemble=2, n=70, seed=9, q=-e0.q, mu_lo=-1.0)]
    f = field_of(wl)
    import torch
    import paper_2403_06706_amd as gcp
    ctx = gcp.Context(device=0, chunk_steps=50)
    ctx.load_field(wl.grid, f, "f64")
    for e in ens:
        ctx.inject(e)
    ctx.advance(1.0, 300)
    ctx.advance(0.5, 200)      # tau = 0.5 on the first step after the change
    ctx.advance(2.0, 100)      # tau = 4
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    of = O.Field(wl.grid, f)
    tab = O.make_ens_table(ens)
    p = np.concatenate([O.inject(of, tab, i, np.arange(e.n, dtype=np.uint32)) for i, e in enumerate(ens)])
    for dt, n in ((1.0, 300), (0.5, 200), (2.0, 100)):
        O.advance(of, tab, p, dt, n)
    compare(st, p, M_ELECTRON, TOL64, "ensembles + variable dt")
    del torch


def test_affine_field_third_order_on_device():
    """On an affine field trilinear interpolation is exact and the right-hand
    side is smooth: the device integration converges at third order in dt."""
    wl = Workload("affine", SphericalGrid(32, 32, 16, 0.1 * AU, 2.0 * AU), lambda g, device=None: fields.affine(g),
                  [Ensemble(n=64, ensemble=0, seed=3, r0=0.8 * AU, lat0=math.radians(10), dlat=math.radians(5),
                            dr0=0.05 * AU, lon0=1.0, dlon=0.5, lambda_par=0.0, r_in=0.15 * AU, r_out=1.9 * AU,
                            mu_lo=-1.0, mu_hi=1.0)], 1.0, 0, "f64", 0)
    f = fields.affine(wl.grid)
    T = 256.0
    fin = {}
    for dt in (0.25, 2.0, 4.0, 8.0, 16.0):
        st, _ = run_gpu(wl, f, n_steps=int(T / dt), dt=dt, order="none")
        assert (st["status"] == 0).all()
        fin[dt] = st
    ref = fin[0.25]
    err = {}
    for dt in (2.0, 4.0, 8.0, 16.0):
        err[dt] = max(np.max(np.abs(fin[dt]["r"] - ref["r"])) / AU, np.max(np.abs(fin[dt]["th"] - ref["th"])),
                      np.max(np.abs(fin[dt]["ph"] - ref["ph"])))
    orders = [math.log2(err[2 * d] / err[d]) for d in (2.0, 4.0, 8.0)]
    say(f"  device observed orders {orders}")
    assert all(2.6 < o < 3.4 for o in orders), (err, orders)
    # and the oracle agrees with the device at every dt
    for dt in (2.0, 16.0):
        p, *_ = run_oracle(wl, f, n_steps=int(T / dt), dt=dt)
        compare(fin[dt], p, M_ELECTRON, TOL64, f"affine dt={dt}")
