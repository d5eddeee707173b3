"""Many ensembles of uneven size in one launch: the graph-captured persistent
push equals the eager grid push bitwise, matches the oracle on sampled
particles of every ensemble, and the autotuner leaves the state untouched."""
import numpy as np
import pytest

import oracle as O
import paper_2403_06706_amd as gcp
from gpu_helpers import compare, same_state, say, stored
from synthetic import AU, M_ELECTRON, SphericalGrid, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batched():
    grid = SphericalGrid(64, 32, 64, 0.1 * AU, 2.0 * AU)
    wl = workloads.config_batched(total=65536, n_ens=16, grid=grid, hours_lo=0.2, hours_hi=0.6)
    f = stored(wl.build_field(grid), "f32")
    return wl, f


def _run(wl, f, steps, graph, **opts):
    import torch
    stream = torch.cuda.Stream() if graph else None
    ctx = gcp.Context(device=0, stream=stream, **opts)
    ctx.load_field(wl.grid, f, "f32")
    for e in wl.ensembles:
        ctx.inject(e)
    if graph:
        with torch.cuda.stream(stream):
            for _ in range(steps // 128):
                ctx.advance_graph(wl.dt, 128)
    else:
        ctx.advance(wl.dt, steps)
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    return st


def test_graph_persistent_equals_eager_and_oracle(batched):
    wl, f = batched
    steps = 2304                                   # longer than every stop time (0.2-0.6 h)
    say(f"batched: {wl.n_particles} electrons in {len(wl.ensembles)} ensembles")
    eager = _run(wl, f, steps, graph=False)
    # pure replays (the device picks no tail form), then the default: replays until the
    # live count read back is below the tail threshold, eager chunks after that
    pers = _run(wl, f, steps, graph=True, persistent=True, tile=512, tail_threshold=0)
    same_state(pers, eager)
    hybrid = _run(wl, f, steps, graph=True, persistent=True, tile=512)
    same_state(hybrid, eager)
    assert (eager["status"] == O.FINISHED).sum() > 1000 and (eager["status"] == O.EXITED).sum() > 1000
    # oracle on 8 sampled ids of every ensemble
    rng = np.random.default_rng(0)
    ids = [np.sort(rng.choice(e.n, size=8, replace=False)).astype(np.uint32) for e in wl.ensembles]
    of = O.Field(wl.grid, f)
    tab = O.make_ens_table(wl.ensembles)
    p = np.concatenate([O.inject(of, tab, i, ids[i]) for i, e in enumerate(wl.ensembles)])
    O.advance(of, tab, p, wl.dt, steps)
    offs = np.cumsum([0] + [e.n for e in wl.ensembles])[:-1]
    gsel = np.concatenate([offs[i] + ids[i] for i in range(len(ids))])
    sub = {k: v[gsel] for k, v in eager.items()}
    compare(sub, p, M_ELECTRON, 1e-6, "batched sample")


def test_autotune_keeps_state_and_applies_options(batched, tmp_path):
    wl, f = batched
    import torch
    ctx = gcp.Context(device=0)
    ctx.load_field(wl.grid, f, "f32")
    for e in wl.ensembles:
        ctx.inject(e)
    ctx.advance(wl.dt, 128)
    before = gcp.state_to_numpy(ctx.get_state())
    cache = str(tmp_path / "tune.json")
    res = ctx.autotune(wl.dt, probe_steps=128, blocks=(64, 128, 256), coarsen=(0, 1), chunks=(64, 128),
                       tiles=(512, 2048), cache=cache, key="batched-test")
    say(f"  autotune: {res}")
    assert res["n_tried"] >= 5 and res["best_rate"] >= res["default_rate"] > 0
    after = gcp.state_to_numpy(ctx.get_state())
    same_state(after, before)
    # continuing with the tuned options gives the same trajectories as the defaults
    ctx.advance(wl.dt, 256)
    tuned = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    ref = gcp.Context(device=0)
    ref.load_field(wl.grid, f, "f32")
    for e in wl.ensembles:
        ref.inject(e)
    ref.advance(wl.dt, 128 + 256)
    plain = gcp.state_to_numpy(ref.get_state())
    ref.close()
    same_state(tuned, plain)
    # a cached choice is applied without timing
    ctx2 = gcp.Context(device=0)
    ctx2.load_field(wl.grid, f, "f32")
    ctx2.inject(wl.ensembles[0])
    res2 = ctx2.autotune(wl.dt, cache=cache, key="batched-test")
    assert res2["cached"] and ctx2.options()["block_size"] == res["options"]["block_size"]
    ctx2.close()
    del torch
