"""Parity at the benchmark sizes, in the launch configurations the benchmark
times, on sampled particles the oracle advances one by one.

* Paper scale: 2^20 electrons in three ensembles on the 256x128x256 FP32
  perturbed-spiral field, FP64 state, cell binning every 64 steps, the tail
  policy on; 2 h of 1 s steps.  64 sampled ids per ensemble.
* Batched: 64 ensembles of uneven size, 4M electrons, the same field, the
  graph-replayed persistent form at tile 512 (one of the autotuner's
  candidates; trajectories are bitwise the same for every tile and workgroup
  size, which test_gpu_order.py checks); 2 h.  4 sampled ids per ensemble.
* Cell binning at the paper scale: the radix sort of 2^20 electrons by cell
  (coarsening 0 and 1) is stable, puts inactive electrons last and sorts on
  the cells of the positions it reorders.
* Network field: 10M electrons through the BF16 network for one 64-step chunk;
  16 sampled ids against the oracle driven by the FP64 network.

Bar: identical status, step and collision counts and relative errors <= 1e-6
in position, u and mu_B for every sampled electron (the oracle reads the same
FP32-rounded field); for the network, positions and u within 3x the errors of
the BF16 arithmetic model (bf16_model.py: the oracle driven by the FP64
network with the device's BF16 roundings) against the oracle driven by the
FP64 network."""
import numpy as np
import pytest

import oracle as O
import paper_2403_06706_amd as gcp
from gpu_helpers import compare, say
from synthetic import M_ELECTRON, workloads

pytestmark = pytest.mark.gpu
STEPS = 7200


@pytest.fixture(scope="module")
def field():
    wl = workloads.config_paper_scale()
    f = wl.build_field(wl.grid, device="cuda")
    return np.ascontiguousarray(f.astype(np.float32).astype(np.float64))


def _sample(st, wl, ids):
    offs = np.cumsum([0] + [e.n for e in wl.ensembles])[:-1]
    gsel = np.concatenate([offs[i] + ids[i] for i in range(len(ids))])
    return {k: v[gsel] for k, v in st.items()}


def _oracle(wl, f, ids, steps):
    of = O.Field(wl.grid, f)
    tab = O.make_ens_table(wl.ensembles)
    p = np.concatenate([O.inject(of, tab, i, ids[i]) for i in range(len(wl.ensembles))])
    O.advance(of, tab, p, wl.dt, steps)
    return p


def test_paper_scale_sampled_parity(field):
    wl = workloads.config_paper_scale()
    say(f"paper scale: {wl.n_particles} electrons, {STEPS} steps")
    ctx = gcp.Context(device=0, precision="f64", order="bin", chunk_steps=64)
    ctx.load_field(wl.grid, field, "f32")
    for e in wl.ensembles:
        ctx.inject(e)
    ctx.advance(wl.dt, STEPS)
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    rng = np.random.default_rng(1)
    ids = [np.sort(rng.choice(e.n, size=64, replace=False)).astype(np.uint32) for e in wl.ensembles]
    p = _oracle(wl, field, ids, STEPS)
    pos, u, mu = compare(_sample(st, wl, ids), p, M_ELECTRON, 1e-6, "paper-scale sample")
    say(f"  sampled {len(p)}: max rel err pos {pos.max():.2e} u {u.max():.2e} mu {mu.max():.2e}; "
        f"active {int((st['status'] == 0).sum())} of {len(st['status'])}")
    assert (st["status"] == O.NONFINITE).sum() == 0
    assert p["k"].sum() > 100 and (st["status"] == O.EXITED).sum() > 1000


def test_batched_full_size_sampled_parity(field):
    import torch
    wl = workloads.config_batched()
    say(f"batched: {wl.n_particles} electrons in {len(wl.ensembles)} ensembles, {STEPS} steps")
    stream = torch.cuda.Stream()
    ctx = gcp.Context(device=0, stream=stream, precision="f64", order="bin", chunk_steps=64, persistent=True,
                      tile=512)
    ctx.load_field(wl.grid, field, "f32")
    for e in wl.ensembles:
        ctx.inject(e)
    with torch.cuda.stream(stream):
        for _ in range(STEPS // 128):
            ctx.advance_graph(wl.dt, 128)
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    rng = np.random.default_rng(2)
    ids = [np.sort(rng.choice(e.n, size=4, replace=False)).astype(np.uint32) for e in wl.ensembles]
    steps = (STEPS // 128) * 128
    p = _oracle(wl, field, ids, steps)
    pos, u, mu = compare(_sample(st, wl, ids), p, M_ELECTRON, 1e-6, "batched sample")
    say(f"  sampled {len(p)}: max rel err pos {pos.max():.2e} u {u.max():.2e} mu {mu.max():.2e}")
    assert (st["status"] == O.NONFINITE).sum() == 0


def test_network_push_full_size_sampled_parity():
    """The network field source at the benchmark's size: 10M electrons, one
    64-step chunk through the BF16 network; 16 sampled electrons advanced by
    the oracle driven by the FP64 network (no scattering, so no decision can
    flip): positions and u within 3x the BF16 model's errors."""
    from dataclasses import replace
    import bf16_model as BM
    from oracle import mlp_oracle as M
    from gpu_helpers import field_of, rel_errors, small
    bf16_round = BM.bf16
    from synthetic import AU
    wl = small(n=64, hours=0.1)
    f = field_of(wl)
    spec = M.make_spec(wl.grid, f, seed=1)
    params = M.init_params(seed=2)
    params["Wo"] = 0.3 * params["Wo"]
    params["co"] = np.array([1.0, 0.3, -0.6, 0.2, 0.8, -0.4])
    params = {k: bf16_round(v) for k, v in params.items()}
    ens = replace(wl.ensembles[0], n=10 << 20, lambda_par=0.0, r_in=0.12 * AU, r_out=1.95 * AU)
    say(f"network push: {ens.n} electrons, 64 steps")
    ctx = gcp.Context(device=0, field_source="mlp", chunk_steps=64)
    ctx.load_field(wl.grid, f, "f64")
    ctx.mlp_set(spec.freq, spec.r_ref, spec.scale, spec.power, params)
    ctx.inject(ens)
    ctx.advance(1.0, 64)
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    rng = np.random.default_rng(3)
    ids = np.sort(rng.choice(ens.n, size=16, replace=False)).astype(np.uint32)
    tab = O.make_ens_table([ens])
    p = O.inject(O.Field(wl.grid, f), tab, 0, ids)

    def cb(r, th, ph):
        return M.field(spec, params, np.array([r]), np.array([th]), np.array([ph]))[0]

    q = p.copy()

    def cb_model(r, th, ph):
        return BM.field(spec, params, np.array([r]), np.array([th]), np.array([ph]))[0]

    O.advance(O.Field(wl.grid, callback=cb), tab, p, 1.0, 64, nthreads=1)
    O.advance(O.Field(wl.grid, callback=cb_model), tab, q, 1.0, 64, nthreads=1)
    sub = {k: v[ids] for k, v in st.items()}
    assert np.array_equal(sub["status"], p["status"]) and np.array_equal(sub["step"], p["step"])
    pos, du, dmu = rel_errors(sub, p, ens.m)
    mq = {"r": q["r"], "th": q["th"], "ph": q["ph"], "u": q["u"], "mu": q["mu_B"] / ens.m}
    pos_m, du_m, _ = rel_errors(mq, p, ens.m)
    say(f"  sampled 16: max position {pos.max():.2e} (model {pos_m.max():.2e}), u {du.max():.2e} "
        f"(model {du_m.max():.2e})")
    assert pos.max() <= BM.MAX_OVER_MODEL * pos_m.max() and du.max() <= BM.MAX_OVER_MODEL * du_m.max()
    assert (st["status"] == O.NONFINITE).sum() == 0


@pytest.mark.parametrize("coarsen", [0, 1])
def test_paper_scale_binning_order(field, coarsen):
    from test_gpu_order import check_binning
    wl = workloads.config_paper_scale()
    ctx = gcp.Context(device=0, precision="f64", order="bin", chunk_steps=64, bin_coarsen=coarsen, tail_threshold=0)
    ctx.load_field(wl.grid, field, "f32")
    for e in wl.ensembles:
        ctx.inject(e)
    check_binning(ctx, wl, coarsen, wl.dt, 1280, "paper scale")
    ctx.close()
