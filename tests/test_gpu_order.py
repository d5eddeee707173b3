"""Reordering, persistence, graphs and checkpoints leave every particle's
trajectory bitwise unchanged (each particle's arithmetic does not depend on
its slot, its neighbours, the chunking or the launch form)."""
import numpy as np
import pytest

import paper_2403_06706_amd as gcp
from gpu_helpers import field_of, run_gpu, same_state, small, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def base():
    wl = small(n=2000, hours=0.5)
    f = field_of(wl)
    st, log = run_gpu(wl, f, order="none", chunk=1800, log_depth=16)
    return wl, f, st, log


@pytest.mark.parametrize("cfg", [
    dict(order="compact", chunk=64),
    dict(order="bin", chunk=64),
    dict(order="bin", chunk=7, coarsen=2),
    dict(order="bin", chunk=1),
    dict(order="bin", chunk=64, block=256),
    dict(order="bin", chunk=64, block=256, tail_threshold=0),
    dict(order="compact", chunk=100, block=128),
    dict(order="bin", chunk=64, persistent=True, tile=256),            # persistent, device picks the quad form
    dict(order="bin", chunk=64, persistent=True, tile=256, tail_threshold=0),                # throughput form only
    dict(order="bin", chunk=64, persistent=True, tile=512, block=256, tail_threshold=4000),  # all pairs, then quad
    dict(order="none", chunk=64, persistent=True, tile=1024, block=128),
    dict(order="bin", chunk=64, tail_threshold=0),             # throughput form and binning every chunk
    dict(order="bin", chunk=64, tail_threshold=1 << 30),       # tail policy once a count has been read back
    dict(order="compact", chunk=16, block=64, tail_threshold=1000),
])
def test_trajectories_invariant(base, cfg):
    wl, f, ref, ref_log = base
    say(f"order invariance {cfg}")
    st, log = run_gpu(wl, f, log_depth=16, **cfg)
    same_state(st, ref)
    assert np.array_equal(log, ref_log)


@pytest.mark.parametrize("precision", ["f32_acc64", "f32_kahan"])
def test_fp32_forms_invariant(base, precision):
    """The FP32-arithmetic forms, FP32 field store: binning every chunk (the
    push applying each reorder's permutation), the tail forms (all pairs, then
    four lanes per particle) and the persistent form give the bits of one
    unreordered launch, the Kahan compensation terms included."""
    wl, f, _, _ = base
    keys = None
    ref, ref_log = run_gpu(wl, f, store_dtype="f32", precision=precision, order="none", chunk=1800, log_depth=16)
    if precision == "f32_kahan":
        keys = list(ref)                 # every field, the compensation terms too
    for cfg in (dict(order="bin", chunk=64), dict(order="bin", chunk=64, tail_threshold=1 << 30),
                dict(order="bin", chunk=64, persistent=True, tile=512, block=256, tail_threshold=4000)):
        say(f"{precision} invariance {cfg}")
        st, log = run_gpu(wl, f, store_dtype="f32", precision=precision, log_depth=16, **cfg)
        same_state(st, ref, keys)
        assert np.array_equal(log, ref_log)


def test_graph_replay_of_the_persistent_form_matches_eager(base):
    """The persistent form in graph replays, the device picking its form from
    the live count: all pairs while all 2,000 electrons are live (tail
    threshold 8,000), four lanes per particle once one has left."""
    wl, f, ref, _ = base
    import torch
    stream = torch.cuda.Stream()
    ctx = gcp.Context(device=0, order="bin", chunk_steps=75, stream=stream, persistent=True, tile=256,
                      tail_threshold=8000)
    ctx.load_field(wl.grid, f, "f64")
    ctx.inject(wl.ensembles[0])
    with torch.cuda.stream(stream):
        ctx.advance_graph(1.0, 150)          # captured and replayed once (no count read back yet)
    c = ctx.counters()
    assert c["form_steps"][1] > 0 and c["form_steps"][2] > 0 and c["form_steps"][0] == 0
    with torch.cuda.stream(stream):
        for _ in range(11):                  # then the eager tail policy (the count read back is below 8,000)
            ctx.advance_graph(1.0, 150)
            stream.synchronize()
            torch.zeros(1000, device="cuda").sum().item()
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    same_state(st, ref)


def test_graph_replay_matches_eager(base):
    wl, f, ref, _ = base
    import torch
    stream = torch.cuda.Stream()
    ctx = gcp.Context(device=0, order="bin", chunk_steps=75, stream=stream, tail_threshold=0)   # replays only
    ctx.load_field(wl.grid, f, "f64")
    ctx.inject(wl.ensembles[0])
    with torch.cuda.stream(stream):
        for _ in range(12):                 # 12 replays of 150 steps = 1800 steps
            ctx.advance_graph(1.0, 150)
            stream.synchronize()
            torch.zeros(1000, device="cuda").sum().item()   # eager work between replays
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    same_state(st, ref)


def test_graph_replays_mixed_with_eager_chunks(base):
    """Eager advances between replays may leave the state in the other buffer
    (an odd number of reorders); the next replay must follow it."""
    wl, f, ref, _ = base
    import torch
    stream = torch.cuda.Stream()
    ctx = gcp.Context(device=0, order="bin", chunk_steps=75, stream=stream, tail_threshold=0)   # replays only
    ctx.load_field(wl.grid, f, "f64")
    ctx.inject(wl.ensembles[0])
    with torch.cuda.stream(stream):
        for n, graph in ((150, True),) * 5 + ((75, False),) + ((150, True),) * 5 + ((225, False),):
            (ctx.advance_graph if graph else ctx.advance)(1.0, n)    # 1800 steps in total
        stream.synchronize()
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    same_state(st, ref)


def test_checkpoint_restore_is_bitwise(base):
    wl, f, ref, _ = base
    import torch
    a = gcp.Context(device=0, chunk_steps=64)
    a.load_field(wl.grid, f, "f64")
    a.inject(wl.ensembles[0])
    a.advance(1.0, 900)
    saved = {k: v.clone() for k, v in a.get_state().items()}
    torch.cuda.synchronize()
    a.close()
    b = gcp.Context(device=0, chunk_steps=50, order="compact")
    b.load_field(wl.grid, f, "f64")
    b.inject(wl.ensembles[0])        # registers the ensemble parameters
    b.set_state(saved)
    b.advance(1.0, 900)
    st = gcp.state_to_numpy(b.get_state())
    b.close()
    same_state(st, ref)


def check_binning(ctx, wl, coarsen, dt, warm_steps, label):
    """Run warm_steps (reordering every chunk), then one more reorder + step,
    and check the reorder against the positions it sorted (shared with the
    full-size test)."""
    ctx.advance(dt, warm_steps)
    order0, _, _ = ctx.get_order(keys=False)          # slot order of the previous reorder
    order0 = order0.cpu().numpy().astype(np.int64)
    snap = gcp.state_to_numpy(ctx.get_state())       # global order: the positions the next reorder sorts
    ctx.advance(dt, 1)
    order1, keys1, live = ctx.get_order()
    order1 = order1.cpu().numpy().astype(np.int64)
    keys1 = keys1.cpu().numpy().view(np.uint32).astype(np.int64)
    n = len(order1)
    say(f"binning {label}: {n} particles, coarsen {coarsen}, {live} live")
    # a permutation of the particles, keys non-decreasing over the slots
    assert np.array_equal(np.sort(order1), np.arange(n))
    assert np.all(np.diff(keys1) >= 0)
    # active particles first, the inactive ones after them
    act = snap["status"][order1] == 0
    assert act[:live].all() and not act[live:].any()
    assert 0 < live < n
    # stable: the new order is numpy's stable sort of the previous slot order by these keys
    key_of = np.empty(n, dtype=np.int64)
    key_of[order1] = keys1
    assert np.array_equal(order1, order0[np.argsort(key_of[order0], kind="stable")])
    # the keys are the cells of the sorted positions (the device decides marginal cases)
    g = wl.grid
    x = (snap["r"] - g.r_min) * ((g.nr - 1) / (g.r_max - g.r_min))
    y = snap["th"] * (g.nth / np.pi) - 0.5
    z = snap["ph"] * (g.nph / (2 * np.pi))
    i = np.clip(np.floor(x), 0, g.nr - 2).astype(np.int64)
    j = np.clip(np.floor(y), 0, g.nth - 2).astype(np.int64)
    k = np.mod(np.floor(z), g.nph).astype(np.int64)
    cdiv = lambda m: (m + (1 << coarsen) - 1) >> coarsen
    want = ((i >> coarsen) * cdiv(g.nth) + (j >> coarsen)) * cdiv(g.nph) + (k >> coarsen)
    want = np.where(snap["status"] == 0, want, cdiv(g.nr) * cdiv(g.nth) * cdiv(g.nph))
    near = lambda v: np.abs(v - np.round(v)) < 1e-9
    marginal = (near(x) | near(y) | near(z)) & (snap["status"] == 0)
    differ = want != key_of
    assert not (differ & ~marginal).any()
    assert differ.sum() <= max(2, n // 100000)
    # the sort is not trivial: many cells, and the order changed
    assert len(np.unique(keys1[:live])) > 10 and (order1 != order0).any()


@pytest.mark.parametrize("coarsen", [0, 1, 2])
def test_binning_sorts_by_cell_stably_inactive_last(coarsen):
    wl = small(n=4096, hours=0.5)
    f = field_of(wl)
    ctx = gcp.Context(device=0, order="bin", chunk_steps=64, bin_coarsen=coarsen, tail_threshold=0)
    ctx.load_field(wl.grid, f, "f64")
    ctx.inject(wl.ensembles[0])
    check_binning(ctx, wl, coarsen, wl.dt, 1280, "small")
    ctx.close()


def test_order_query_states():
    wl = small(n=300, hours=0.01)
    f = field_of(wl)
    ctx = gcp.Context(device=0, order="compact", chunk_steps=16)
    ctx.load_field(wl.grid, f, "f64")
    ctx.inject(wl.ensembles[0])
    with pytest.raises(gcp.GCError):
        ctx.get_order()                      # no reorder since the injection
    ctx.advance(1.0, 16)
    with pytest.raises(gcp.GCError):
        ctx.get_order()                      # a compaction has no cell keys ...
    gid, key, live = ctx.get_order(keys=False)   # ... but a slot order
    assert key is None and sorted(gid.cpu().tolist()) == list(range(300)) and live == 300
    ctx.close()


def test_counters_count_active_steps(base):
    wl, f, ref, _ = base
    ctx = gcp.Context(device=0, timing=True)
    ctx.load_field(wl.grid, f, "f64")
    ctx.inject(wl.ensembles[0])
    ctx.advance(1.0, 1800)
    c = ctx.counters()
    ctx.close()
    assert c["particle_steps"] == int(ref["step"].sum())
    assert c["n_push"] == (1800 + 63) // 64 and c["push_ms"] > 0
    assert c["n_reorder"] > 0 and c["reorder_ms"] > 0
    # timing 2: the push launches only
    ctx = gcp.Context(device=0, timing="push")
    ctx.load_field(wl.grid, f, "f64")
    ctx.inject(wl.ensembles[0])
    ctx.advance(1.0, 1800)
    c2 = ctx.counters()
    ctx.close()
    assert c2["particle_steps"] == c["particle_steps"] and c2["n_push"] == c["n_push"] and c2["push_ms"] > 0
    assert c2["n_reorder"] == 0 and c2["reorder_ms"] == 0
