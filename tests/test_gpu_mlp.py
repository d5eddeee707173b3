"""Neural field on the device against the FP64 NumPy oracle of the network:
point evaluation (B, E, grad|B|, (b.grad)b), the training loss and its
gradient, one optimizer step, the push with the network as field source; then
training on samples drawn along trajectories, judged against the grid.

The device multiplies in BF16 with FP32 accumulation.  The test networks have
BF16-representable weights (rounded on the host before upload), so that the
device's BF16 weight copy is exact and the remaining difference is the BF16
rounding of the activations and tangents (at most 2^-8 of each value) plus
FP32 features and accumulation.  Every tolerance comes from the arithmetic
model in bf16_model.py, evaluated on the CPU from the oracle's network: the
oracle's network with the device's BF16 rounding points.  The device must stay
within a small multiple of the model's error (3x its maximum, 2x its RMS,
3x its relative gradient error); no bar is set from device output."""
import math
from dataclasses import replace

import numpy as np
import pytest

import bf16_model as BM
import oracle as O
from gpu_helpers import field_of, oracle_to_state, rel_errors, say, small
from oracle import mlp_oracle as M
from synthetic import AU

pytestmark = pytest.mark.gpu
bf16_round = BM.bf16


@pytest.fixture(scope="module")
def net():
    import torch
    import paper_2403_06706_amd as gcp
    wl = small(n=64, hours=0.1)
    f = field_of(wl)
    spec = M.make_spec(wl.grid, f, seed=1)
    params = M.init_params(seed=2)
    # outputs biased away from zero (|B| and |E| never vanish), random variation of about 0.3
    params["Wo"] = 0.3 * params["Wo"]
    params["co"] = np.array([1.0, 0.3, -0.6, 0.2, 0.8, -0.4])
    params = {k: bf16_round(v) for k, v in params.items()}
    ctx = gcp.Context(device=0)
    ctx.load_field(wl.grid, f, "f64")
    ctx.mlp_set(spec.freq, spec.r_ref, spec.scale, spec.power, params)
    yield ctx, wl, f, spec, params
    ctx.close()
    torch.cuda.synchronize()


def _points(rng, n):
    return np.stack([rng.uniform(0.15, 1.9, n) * AU, rng.uniform(0.3, math.pi - 0.3, n),
                     rng.uniform(-1.0, 7.0, n)])


@pytest.fixture(scope="module")
def eval_bars(net):
    """(max, rms) bars per vector from the arithmetic model at 4,096 points."""
    _, _, _, spec, params = net
    bars = BM.eval_bars(spec, params, _points(np.random.default_rng(5), 4096))
    say("evaluation bars from the BF16 model: " + ", ".join(f"{k} {v[0]:.2e}/{v[1]:.2e}" for k, v in bars.items()))
    return bars


def test_parameters_round_trip(net):
    ctx, wl, f, spec, params = net
    back = ctx.mlp_params()
    for k, v in params.items():
        assert np.array_equal(back[k].astype(np.float64), v.astype(np.float32).astype(np.float64)), k


@pytest.mark.parametrize("n", [1, 63, 1000, 4096 + 17])
def test_eval_matches_oracle(net, eval_bars, n):
    import torch
    ctx, wl, f, spec, params = net
    rng = np.random.default_rng(11 + n)
    pts = _points(rng, n)
    got = ctx.mlp_eval(torch.tensor(pts, device="cuda")).cpu().numpy()
    ref = M.field(spec, params, pts[0], pts[1], pts[2])
    assert np.all(np.isfinite(got))
    # per-point scales: |B|, |E|; the Jacobian norm of B in the local basis for
    # grad|B|; that norm over |B| plus 1/r (field-line curvature scale) for K
    errs = BM.field_errors(got, ref, BM.field_scales(spec, params, pts, ref))
    for name, err in errs.items():
        rms = np.sqrt(np.mean(err ** 2))
        say(f"eval n={n} {name}: max {err.max():.2e} rms {rms:.2e} (bars {eval_bars[name][0]:.2e} / "
            f"{eval_bars[name][1]:.2e})")
        assert err.max() <= eval_bars[name][0], (name, err.max())
        if n >= 1000:            # an RMS over few points says little
            assert rms <= eval_bars[name][1], (name, rms)


def _pairs(spec, rng, npair):
    p1 = _points(rng, npair).T
    p2 = p1 + np.stack([rng.normal(0, 0.02 * AU, npair), rng.normal(0, 0.02, npair),
                        rng.normal(0, 0.02, npair)], axis=1)
    env1, _ = M.envelope(spec, p1[:, 0])
    env2, _ = M.envelope(spec, p2[:, 0])
    t1 = rng.normal(0, 1, (npair, 6)) * env1
    t2 = (t1 / env1 + rng.normal(0, 0.1, (npair, 6))) * env2
    return p1, p2, t1, t2


def test_training_gradient_matches_oracle(net):
    import torch
    ctx, wl, f, spec, params = net
    rng = np.random.default_rng(21)
    npair = 333
    p1, p2, t1, t2 = _pairs(spec, rng, npair)
    wc = np.array([1.0, 0.5, 1.0, 2.0, 1.0, 0.5])
    beta = 4.0
    P = torch.tensor(np.concatenate([p1, p2]).T.copy(), device="cuda")
    T = torch.tensor(np.concatenate([t1, t2]), device="cuda")
    loss = ctx.mlp_train_step(P, T, wc=wc, beta_pair=beta, apply=False)
    g = ctx.mlp_grads()
    L, gref = M.loss_and_grad(spec, params, p1, t1, p2, t2, wc, beta)
    Lm, gmod = BM.loss_and_grad(spec, params, p1, t1, p2, t2, wc, beta)
    # bars: 3x the model's error, plus FP32 accumulation over the 2 x 333 rows
    # (the device's partial sums in another order: rows x 2^-24, doubled)
    fp32 = 2 * (2 * npair) * 2.0 ** -24
    say(f"loss device {loss:.6e} oracle {L:.6e} model {Lm:.6e}")
    assert abs(loss - L) <= BM.MAX_OVER_MODEL * abs(Lm - L) + fp32 * L
    for k in gref:
        a, b, m = g[k].astype(np.float64).ravel(), gref[k].ravel(), gmod[k].ravel()
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        rel_m = np.linalg.norm(m - b) / np.linalg.norm(b)
        bar = BM.MAX_OVER_MODEL * rel_m + fp32
        say(f"grad {k}: rel {rel:.2e} (model {rel_m:.2e}, bar {bar:.2e})")
        assert rel <= bar, (k, rel, bar)
    # the parameters did not move (apply = 0)
    back = ctx.mlp_params()
    assert all(np.array_equal(back[k].astype(np.float64), params[k]) for k in params)


def test_adam_step_follows_the_oracle_gradient(net):
    """One Adam step from zero moments moves every parameter by lr * g / (|g| +
    eps') (Kingma & Ba, bias-corrected): about lr against the sign of g where |g|
    is well above the device's gradient error."""
    import torch
    import paper_2403_06706_amd as gcp
    ctx0, wl, f, spec, params = net
    ctx = gcp.Context(device=0)
    ctx.load_field(wl.grid, f, "f64")
    ctx.mlp_set(spec.freq, spec.r_ref, spec.scale, spec.power, params)
    rng = np.random.default_rng(31)
    p1, p2, t1, t2 = _pairs(spec, rng, 256)
    P = torch.tensor(np.concatenate([p1, p2]).T.copy(), device="cuda")
    T = torch.tensor(np.concatenate([t1, t2]), device="cuda")
    lr = 1e-3
    ctx.mlp_train_step(P, T, beta_pair=1.0, lr=lr, step=1, apply=True)
    after = ctx.mlp_params()
    ctx.close()
    _, gref = M.loss_and_grad(spec, params, p1, t1, p2, t2, np.ones(6), 1.0)
    for k in gref:
        d = after[k].astype(np.float64) - params[k]
        g = gref[k]
        assert np.all(np.abs(d) <= lr * (1 + 1e-3) + 1e-7 * np.abs(params[k])), k
        big = np.abs(g) > 0.1 * np.abs(g).max()
        assert np.all(np.sign(d[big]) == -np.sign(g[big])), k
        assert np.allclose(np.abs(d[big]), lr, rtol=1e-2, atol=1e-7 * np.abs(params[k][big]).max()), k


def test_push_with_network_matches_oracle(net):
    """Same particles, no scattering (no branch to flip): the device push with
    the network as field source against the oracle driven by the FP64 network."""
    import paper_2403_06706_amd as gcp
    _, wl, f, spec, params = net
    ens = replace(wl.ensembles[0], n=48, lambda_par=0.0, r_in=0.12 * AU, r_out=1.95 * AU)
    of = O.Field(wl.grid, f)
    tab = O.make_ens_table([ens])
    p = O.inject(of, tab, 0, np.arange(ens.n, dtype=np.uint32))
    ctx = gcp.Context(device=0, field_source="mlp")
    ctx.load_field(wl.grid, f, "f64")
    ctx.mlp_set(spec.freq, spec.r_ref, spec.scale, spec.power, params)
    ctx.inject(ens)
    ctx.set_state(oracle_to_state(p, ens.m))
    n_steps = 240
    ctx.advance(1.0, n_steps)
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()

    def cb(r, th, ph):
        return M.field(spec, params, np.array([r]), np.array([th]), np.array([ph]))[0]

    # the arithmetic model: the oracle integrator driven by the BF16-rounded network
    q = p.copy()

    def cb_model(r, th, ph):
        return BM.field(spec, params, np.array([r]), np.array([th]), np.array([ph]))[0]

    O.advance(O.Field(wl.grid, callback=cb), tab, p, 1.0, n_steps, nthreads=1)
    O.advance(O.Field(wl.grid, callback=cb_model), tab, q, 1.0, n_steps, nthreads=1)
    assert np.all(p["status"] == O.ACTIVE)
    assert np.array_equal(st["status"], p["status"])
    assert np.array_equal(st["step"], p["step"])
    pos, du, dmu = rel_errors(st, p, ens.m)
    mq = {k: q[k] for k in ("r", "th", "ph", "u")}
    mq["mu"] = q["mu_B"] / ens.m
    pos_m, du_m, _ = rel_errors(mq, p, ens.m)
    say(f"network push: max position {pos.max():.2e} (model {pos_m.max():.2e}), u {du.max():.2e} "
        f"(model {du_m.max():.2e}), mu {dmu.max():.2e}")
    assert pos.max() <= BM.MAX_OVER_MODEL * pos_m.max()
    assert du.max() <= BM.MAX_OVER_MODEL * du_m.max()
    assert dmu.max() == 0.0          # no collision: mu_B is never touched
