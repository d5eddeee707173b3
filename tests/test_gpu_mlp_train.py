"""Training of the neural field on samples drawn along trajectories of the
small spiral workload (8,192 electrons, 2 h, positions every 16 steps), by the
library's own forward and backward kernels, and what the trained network gains
over the method without it.

Gain: the network (GC_MLP_PARAMS BF16 weights, 200 KB) reproduces the field it
learned from with 1/32 of the 64x32x64 grid's memory, and electrons pushed
through it stay as close to electrons pushed through the closed-form spiral as
those pushed through the grid do; a trilinear grid of the network's own memory
footprint is several times further off, in the field and in the trajectories.
The closed-form spiral (oracle) is the truth for both."""
import math
from dataclasses import replace

import numpy as np
import pytest

import oracle as O
from gpu_helpers import oracle_to_state, rel_errors, say
from synthetic import AU, B0_1AU, OMEGA_SUN, V_WIND, SphericalGrid, fields, workloads
from synthetic.mlp_setup import init_params, make_spec

pytestmark = pytest.mark.gpu

A0 = B0_1AU * AU * AU
PARKER = {"a0": A0, "omega": OMEGA_SUN, "v_wind": V_WIND}
COARSE = (24, 12, 16)          # a grid of about the network's footprint (235 KB in FP32)


@pytest.fixture(scope="module")
def trained():
    import torch
    import paper_2403_06706_amd as gcp
    from paper_2403_06706_amd import neural
    wl = workloads.config_small(n=8192)
    f = fields.parker(wl.grid)
    ctx = gcp.Context(device=0)
    ctx.load_field(wl.grid, f, "f64")
    ctx.inject(wl.ensembles[0])
    pos = neural.collect_positions(ctx, 1.0, wl.n_steps, every=16)
    spec = make_spec(wl.grid, f, seed=1)
    ctx.mlp_set(spec.freq, spec.r_ref, spec.scale, spec.power, init_params(seed=4))
    held = gcp.Context(device=0)
    held.load_field(wl.grid, f, "f64")
    held.inject(replace(wl.ensembles[0], n=1024, seed=7))
    hold = neural.collect_positions(held, 1.0, wl.n_steps, every=64)
    held.close()
    g = wl.grid
    sigma = [0.1 * (g.r_max - g.r_min) / (g.nr - 1), 0.1 * math.pi / g.nth, 0.1 * 2 * math.pi / g.nph]
    say(f"training on {pos.shape[1]} trajectory positions")
    losses = neural.train(ctx, pos, steps=3000, n_pairs=8192, sigma=sigma, beta_pair=100.0, lr=2e-3, seed=0)
    torch.cuda.synchronize()
    yield dict(ctx=ctx, wl=wl, f=f, spec=spec, pos=pos, hold=hold, losses=losses)
    ctx.close()


def test_training_converges_and_fits_the_grid(trained):
    from paper_2403_06706_amd import neural
    losses = np.array(trained["losses"])
    say(f"loss {losses[0]:.3e} -> {losses[-1]:.3e} over {len(losses)} steps "
        f"({len(losses) * 8192 * 2 / 1e6:.0f}M samples)")
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 1e-3 * losses[0]
    assert np.mean(losses[-100:]) < np.mean(losses[1000:1100])
    e = neural.field_errors(trained["ctx"], trained["hold"])
    say(f"held-out field error against the grid: {e}")
    # measured on MI355X: B 7e-4, E 5e-4, grad|B| 1.4e-2, K 5e-3
    assert e["B"] <= 2e-3 and e["E"] <= 2e-3 and e["G"] <= 3e-2 and e["K"] <= 1e-2


def _truth(pts):
    return np.stack([O.parker_closed_form(A0, OMEGA_SUN, V_WIND, pts[0, i], pts[1, i]) for i in range(pts.shape[1])])


def _vs_truth(v, truth):
    out = {}
    for name, sl in (("B", slice(0, 3)), ("E", slice(3, 6)), ("G", slice(6, 9)), ("K", slice(9, 12))):
        num = np.linalg.norm(v[:, sl] - truth[:, sl], axis=1)
        out[name] = float(np.sqrt(np.mean((num / np.linalg.norm(truth[:, sl], axis=1)) ** 2)))
    return out


def test_network_matches_grid_accuracy_at_a_thirtieth_of_its_memory(trained):
    import paper_2403_06706_amd as gcp
    ctx, wl = trained["ctx"], trained["wl"]
    H = trained["hold"][:, :20000].contiguous()
    truth = _truth(H.cpu().numpy())
    net = _vs_truth(ctx.mlp_eval(H).cpu().numpy(), truth)
    fine = _vs_truth(ctx.field_sample(H).cpu().numpy(), truth)
    cg = SphericalGrid(*COARSE, wl.grid.r_min, wl.grid.r_max)
    c = gcp.Context(device=0)
    c.load_field(cg, fields.parker(cg), "f32")
    coarse = _vs_truth(c.field_sample(H).cpu().numpy(), truth)
    c.close()
    net_bytes = gcp.GC_MLP_PARAMS * 2
    fine_bytes = wl.grid.nr * wl.grid.nth * (wl.grid.nph + 1) * 12 * 4
    coarse_bytes = cg.nr * cg.nth * (cg.nph + 1) * 12 * 4
    say(f"vs closed form: network ({net_bytes} B) {net}; grid ({fine_bytes} B) {fine}; "
        f"equal-memory grid ({coarse_bytes} B) {coarse}")
    assert fine_bytes >= 30 * net_bytes and coarse_bytes <= 1.2 * net_bytes
    assert net["B"] <= 1.2 * fine["B"] and net["E"] <= 1.5 * fine["E"]
    assert coarse["B"] >= 4 * net["B"] and coarse["E"] >= 4 * net["E"] and coarse["G"] >= 2 * net["G"]


def test_trajectories_through_the_network_stay_with_the_closed_form(trained):
    """256 electrons without scattering for 2000 s (they reach the outer shell
    after about 2500 s), started from the same oracle-injected state."""
    import paper_2403_06706_amd as gcp
    ctx, wl, f, spec = trained["ctx"], trained["wl"], trained["f"], trained["spec"]
    ens = replace(wl.ensembles[0], n=256, lambda_par=0.0, seed=11, r_in=0.12 * AU)
    tab = O.make_ens_table([ens])
    p0 = O.inject(O.Field(wl.grid, f), tab, 0, np.arange(ens.n, dtype=np.uint32))
    truth = p0.copy()
    O.advance(O.Field(wl.grid, parker=PARKER), tab, truth, 1.0, 2000)
    params = ctx.mlp_params()

    def run(grid, data, store, source):
        c = gcp.Context(device=0, field_source=source)
        c.load_field(grid, data, store)
        if source == "mlp":
            c.mlp_set(spec.freq, spec.r_ref, spec.scale, spec.power, params)
        c.inject(ens)
        c.set_state(oracle_to_state(p0, ens.m))
        c.advance(1.0, 2000)
        st = gcp.state_to_numpy(c.get_state())
        c.close()
        assert np.array_equal(st["status"], truth["status"]) and np.all(truth["status"] == O.ACTIVE)
        return np.median(rel_errors(st, truth, ens.m)[0])

    cg = SphericalGrid(*COARSE, wl.grid.r_min, wl.grid.r_max)
    e_grid = run(wl.grid, f, "f64", "grid")
    e_net = run(wl.grid, f, "f64", "mlp")
    e_coarse = run(cg, fields.parker(cg), "f32", "grid")
    say(f"median position error after 2000 s vs closed form: grid {e_grid:.2e}, network {e_net:.2e}, "
        f"equal-memory grid {e_coarse:.2e}")
    # measured on MI355X: grid 1.6e-3, network 1.1e-3, equal-memory grid 1.4e-2
    assert e_net <= 1.2 * e_grid
    assert e_coarse >= 5 * e_net
