"""Device memory from the caller's allocator (gc_options.dev_alloc / dev_free):
with torch's caching allocator behind it (the binding's default) the
context's state, field and scratch buffers show up in torch's accounting, are
returned on destruction, and the results are bitwise those of the
hipMalloc-backed context (allocator "hip")."""
import numpy as np
import pytest

import paper_2403_06706_amd as gcp
from gpu_helpers import field_of, same_state, small

pytestmark = pytest.mark.gpu


def _run(wl, f, allocator):
    ctx = gcp.Context(device=0, allocator=allocator, log_depth=16)
    ctx.load_field(wl.grid, f, "f32")
    for e in wl.ensembles:
        ctx.inject(e)
    ctx.advance(wl.dt, wl.n_steps)
    st = gcp.state_to_numpy(ctx.get_state())
    log = ctx.get_log().cpu().numpy()
    return ctx, st, log


def test_torch_allocator_backs_the_context():
    import torch
    wl = small(n=4096, hours=0.5)
    f = field_of(wl)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(0)
    ctx, st_t, log_t = _run(wl, f, "torch")
    held = torch.cuda.memory_allocated(0) - before
    packed = wl.grid.nr * wl.grid.nth * (wl.grid.nph + 1) * 12 * 4
    assert held >= packed + 4096 * 176            # field and two state buffers at least
    ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) - before < held // 4      # returned (outputs above are host copies)
    ctx2, st_h, log_h = _run(wl, f, "hip")
    ctx2.close()
    same_state(st_t, st_h)
    assert np.array_equal(log_t, log_h)


def test_allocator_choice_is_checked():
    with pytest.raises(ValueError):
        gcp.Context(device=0, allocator="bogus")


def test_torch_allocator_is_the_default():
    import torch
    wl = small(n=512, hours=0.01)
    f = field_of(wl)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(0)
    with gcp.Context(device=0) as ctx:
        ctx.load_field(wl.grid, f, "f32")
        assert torch.cuda.memory_allocated(0) - before >= wl.grid.nr * wl.grid.nth * (wl.grid.nph + 1) * 12 * 4
