"""Moments kernel against the oracle's moments of the same particle state.
The state is made by the oracle (injection and 3600 steps) and loaded into the
device with gc_set_state.  Counts and histograms must match exactly; each
fixed-point sum may differ by at most one unit per particle (floor of a product
computed in a different rounding order)."""
import numpy as np
import pytest

import oracle as O
import paper_2403_06706_amd as gcp
from gpu_helpers import field_of, oracle_to_state, run_oracle, small, say, state_to_oracle, stored
from synthetic import AU, E_CHARGE

pytestmark = pytest.mark.gpu

SPEC = dict(n_rbins=38, r_lo=0.1 * AU, r_hi=2.0 * AU, n_mubins=20, sel_r_lo=0.9 * AU, sel_r_hi=1.1 * AU,
            age_lo=0.0, age_hi=1e9, min_collisions=1, n_agebins=6, age_max=3600.0, n_ebins=40, e_lo=79e3,
            e_hi=83e3, e_unit=E_CHARGE, len_unit=AU)


def _check(got, want, spec):
    assert got.shape == want.shape
    nr = spec.n_rbins
    fixed = np.zeros(len(want), dtype=bool)
    fixed[6] = True
    fixed[8 + 1:8 + 3 * nr:3] = True
    fixed[8 + 2:8 + 3 * nr:3] = True
    assert np.array_equal(got[~fixed], want[~fixed])
    active = int(want[0])
    assert np.all(np.abs(got[fixed] - want[fixed]) <= active)


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_moments_match_oracle(store):
    wl = small(n=5000, hours=1.0)
    f = stored(field_of(wl), store)
    p, _, of, tab = run_oracle(wl, f, n_steps=3600, dt=1.0)
    spec = O.MomentSpec(**SPEC)
    want = O.moments(of, tab, p, spec)
    ctx = gcp.Context(device=0)
    ctx.load_field(wl.grid, f, store)
    ctx.inject(wl.ensembles[0])             # registers the ensemble parameters
    ctx.set_state(oracle_to_state(p, wl.ensembles[0].m))
    got = ctx.moments(spec).cpu().numpy()
    ctx.close()
    say(f"  moments counts {want[:8]}")
    _check(got, want, spec)
    assert want[8 + 3 * spec.n_rbins:].sum() > 100          # the histograms are populated


@pytest.mark.parametrize("order", ["bin", "compact"])
def test_moments_after_reorders_equal_the_oracle_of_the_device_state(order):
    """After reorders have moved exited electrons past the live prefix, the
    device reads only that prefix and adds the sums the reorders kept for the
    slots past it: each snapshot, and their accumulated sum, must equal the
    oracle's moments of the device's own state."""
    import torch
    wl = small(n=5000, hours=1.0)
    f = stored(field_of(wl), "f64")
    spec = O.MomentSpec(**SPEC)
    of = O.Field(wl.grid, f)
    tab = O.make_ens_table(wl.ensembles)
    ctx = gcp.Context(device=0, order=order, chunk_steps=64)
    ctx.load_field(wl.grid, f, "f64")
    ctx.inject(wl.ensembles[0])
    acc = torch.zeros(ctx.moments_size(spec), dtype=torch.int64, device="cuda:0")
    want_sum = None
    for rnd in range(3):
        ctx.advance(wl.dt, 64 * 20)
        got = ctx.moments(spec).cpu().numpy()
        ctx.moments(spec, out=acc, accumulate=True)
        p = state_to_oracle(gcp.state_to_numpy(ctx.get_state()), wl.ensembles[0].m)
        want = O.moments(of, tab, p, spec)
        say(f"  {order} snapshot {rnd}: counts {want[:8]}")
        _check(got, want, spec)
        want_sum = want if want_sum is None else want_sum + want
    ctx.close()
    assert want[1] > 0 and want[0] > 0          # exited electrons past the prefix, active ones in it
    got_sum = acc.cpu().numpy()
    nr = spec.n_rbins
    fixed = np.zeros(len(want_sum), dtype=bool)
    fixed[6] = True
    fixed[8 + 1:8 + 3 * nr:3] = True
    fixed[8 + 2:8 + 3 * nr:3] = True
    assert np.array_equal(got_sum[~fixed], want_sum[~fixed])
    assert np.all(np.abs(got_sum[fixed] - want_sum[fixed]) <= 3 * 5000)
