"""Neural field on the device against the FP64 NumPy oracle of the network:
point evaluation (B, E, grad|B|, (b.grad)b), the training loss and its
gradient, one optimizer step, the push with the network as field source; then
training on samples drawn along trajectories, judged against the grid.

The device multiplies in BF16 with FP32 accumulation.  The test networks have
BF16-representable weights (rounded on the host before upload), so that the
device's BF16 weight copy is exact and the remaining difference is the BF16
rounding of the activations and tangents (relative 2^-9 per value) plus FP32
features and accumulation.  Rounding errors of 2^-9 in sums of 128 terms of
random sign partly cancel: the outputs come out at a few 1e-4 of their size
(RMS).  Derivative quantities are judged against the Jacobian norm of B (for
grad|B|, which is a projection of it) and that norm over |B| plus 1/r (for the
curvature (b.grad)b); the tolerances are 3-4x the errors measured on MI355X."""
import math
from dataclasses import replace

import numpy as np
import pytest

import oracle as O
from gpu_helpers import field_of, oracle_to_state, rel_errors, say, small
from oracle import mlp_oracle as M
from synthetic import AU

pytestmark = pytest.mark.gpu


def bf16_round(a):
    """Nearest BF16-representable values (round half to even), as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


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


def test_parameters_round_trip(net):
    ctx, wl, f, spec, params = net
    back = ctx.mlp_params()
    for k, v in params.items():
        assert np.array_equal(back[k].astype(np.float64), v.astype(np.float32).astype(np.float64)), k


@pytest.mark.parametrize("n", [1, 63, 1000, 4096 + 17])
def test_eval_matches_oracle(net, n):
    import torch
    ctx, wl, f, spec, params = net
    rng = np.random.default_rng(11 + n)
    pts = _points(rng, n)
    got = ctx.mlp_eval(torch.tensor(pts, device="cuda")).cpu().numpy()
    ref = M.field(spec, params, pts[0], pts[1], pts[2])
    assert np.all(np.isfinite(got))
    # per-point scales: |B|, |E|; the Jacobian norm of B in the local basis for
    # grad|B|; that norm over |B| plus 1/r (field-line curvature scale) for K
    r, th = pts[0], pts[1]
    h0, dh0 = M.features(spec, pts[0], pts[1], pts[2])
    y, dy = M.forward_jvp(params, h0, dh0)
    env, denv = M.envelope(spec, r)
    J = np.stack([denv[:, :3] * y[:, :3] + env[:, :3] * dy[0][:, :3], env[:, :3] * dy[1][:, :3] / r[:, None],
                  env[:, :3] * dy[2][:, :3] / (r * np.sin(th))[:, None]])
    jn = np.sqrt(np.sum(J ** 2, axis=(0, 2)))
    bn = np.linalg.norm(ref[:, 0:3], axis=1)
    scales = {"B": bn, "E": np.linalg.norm(ref[:, 3:6], axis=1), "G": jn, "K": jn / bn + 1.0 / r}
    tol = {"B": (4e-3, 1e-3), "E": (4e-3, 1e-3), "G": (4e-2, 6e-3), "K": (1.5e-2, 3e-3)}   # (max, rms)
    for name, sl in (("B", slice(0, 3)), ("E", slice(3, 6)), ("G", slice(6, 9)), ("K", slice(9, 12))):
        err = np.linalg.norm(got[:, sl] - ref[:, sl], axis=1) / scales[name]
        say(f"eval n={n} {name}: max {err.max():.2e} rms {np.sqrt(np.mean(err ** 2)):.2e}")
        assert err.max() <= tol[name][0], (name, err.max())
        assert np.sqrt(np.mean(err ** 2)) <= tol[name][1], name


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
    say(f"loss device {loss:.6e} oracle {L:.6e}")
    assert abs(loss - L) <= 1e-3 * L
    for k in gref:
        a, b = g[k].astype(np.float64).ravel(), gref[k].ravel()
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        say(f"grad {k}: rel {rel:.2e} cos {cos:.6f}")
        assert rel <= 2e-2 and cos >= 0.9998, (k, rel, cos)
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

    O.advance(O.Field(wl.grid, callback=cb), tab, p, 1.0, n_steps, nthreads=1)
    assert np.all(p["status"] == O.ACTIVE)
    assert np.array_equal(st["status"], p["status"])
    assert np.array_equal(st["step"], p["step"])
    pos, du, dmu = rel_errors(st, p, ens.m)
    say(f"network push: max position {pos.max():.2e}, u {du.max():.2e}, mu {dmu.max():.2e}")
    assert pos.max() <= 1e-4
    assert du.max() <= 3e-4
    assert dmu.max() == 0.0          # no collision: mu_B is never touched
