"""The training step that allocates nothing (gc_mlp_train_step_noalloc, its
workspace in the library's static device array) against the allocating one
(gc_mlp_train_step) on the same network and points: two calls in a row, the
second with fewer pairs, each giving bitwise the same loss, gradient and
updated parameters; no device memory is taken during the call; more pairs
than the array holds are refused."""
import math

import numpy as np
import pytest

from gpu_helpers import say
from synthetic import workloads
from synthetic.mlp_setup import init_params, make_spec

pytestmark = pytest.mark.gpu
MAX_PAIRS = 2048


def _points(wl, n, seed):
    """n random pairs inside the grid (partners displaced by about a tenth of a cell)."""
    import torch
    rng = np.random.default_rng(seed)
    g = wl.grid
    r = rng.uniform(g.r_min + 0.05 * (g.r_max - g.r_min), g.r_max - 0.05 * (g.r_max - g.r_min), n)
    th = rng.uniform(0.6, math.pi - 0.6, n)
    ph = rng.uniform(0.0, 2 * math.pi, n)
    d = [0.1 * (g.r_max - g.r_min) / (g.nr - 1), 0.1 * math.pi / g.nth, 0.1 * 2 * math.pi / g.nph]
    p2 = [r + rng.normal(0, d[0], n), th + rng.normal(0, d[1], n), ph + rng.normal(0, d[2], n)]
    pts = np.stack([np.concatenate([a, b]) for a, b in zip((r, th, ph), p2)])
    return torch.tensor(pts, dtype=torch.float64, device="cuda").contiguous()


@pytest.fixture(scope="module")
def pair():
    import paper_2403_06706_amd as gcp
    wl = workloads.config_small(n=16)
    f = wl.build_field(wl.grid)
    spec = make_spec(wl.grid, f, seed=1)
    params = init_params(seed=4)
    ctxs = []
    for _ in range(2):
        c = gcp.Context(device=0)
        c.load_field(wl.grid, f, "f64")
        c.mlp_set(spec.freq, spec.r_ref, spec.scale, spec.power, params)
        ctxs.append(c)
    yield wl, ctxs[0], ctxs[1]
    for c in ctxs:
        c.close()


def _same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k]), f"{what} {k} differs"


@pytest.mark.parametrize("n_pairs,step", [(MAX_PAIRS, 1), (300, 2)])
def test_noalloc_step_matches_the_allocating_step(pair, n_pairs, step):
    import torch
    wl, ref, dut = pair
    pts = _points(wl, n_pairs, seed=step)
    tgt = ref.field_sample(pts)[:, :6].contiguous()
    kw = dict(beta_pair=50.0, lr=1e-3, step=step, apply=True)
    say(f"no-alloc training step: {n_pairs} pairs, Adam step {step}")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(0)
    loss_d = dut.mlp_train_step(pts, tgt, noalloc=True, **kw)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == before          # nothing taken from the allocator
    loss_r = ref.mlp_train_step(pts, tgt, **kw)
    say(f"  loss {loss_d:.6e} (allocating step {loss_r:.6e})")
    assert math.isfinite(loss_d) and loss_d > 0
    assert loss_d == loss_r
    _same(dut.mlp_grads(), ref.mlp_grads(), "gradient")
    _same(dut.mlp_params(), ref.mlp_params(), "updated parameter")


def test_noalloc_step_refuses_more_pairs_than_the_array_holds(pair):
    import paper_2403_06706_amd as gcp
    wl, _, dut = pair
    pts = _points(wl, MAX_PAIRS + 1, seed=9)
    tgt = dut.field_sample(pts)[:, :6].contiguous()
    before = dut.mlp_params()
    with pytest.raises(gcp.GCError, match="n_pairs must be in"):
        dut.mlp_train_step(pts, tgt, noalloc=True, step=3)
    _same(dut.mlp_params(), before, "parameter after a refused call")
