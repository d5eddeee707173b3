"""Neural-field workflow on the device: sample positions along trajectories,
train the network on the gridded field at those positions, judge it against
the grid.  Orchestration only: the forward and backward passes, the optimizer
and both field evaluations run in the library's kernels (gc_mlp_train_step,
gc_mlp_eval, gc_field_sample); torch draws the batch indices and the pair
offsets and slices device buffers.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional

from . import GC_ACTIVE


def collect_positions(ctx, dt: float, n_steps: int, every: int, max_points: Optional[int] = None):
    """Advance the context's particles by n_steps (in chunks of `every`) and
    return the positions (r, th, ph) of the active particles after each chunk
    as a device float64 tensor [3, M]."""
    import torch
    chunks = []
    done, total = 0, 0
    while done < n_steps:
        k = min(every, n_steps - done)
        ctx.advance(dt, k)
        done += k
        st = ctx.get_state()
        live = st["status"] == GC_ACTIVE
        pos = torch.stack([st["r"][live], st["th"][live], st["ph"][live]])
        chunks.append(pos)
        total += pos.shape[1]
        if max_points is not None and total >= max_points:
            break
    out = torch.cat(chunks, dim=1).contiguous()
    return out[:, :max_points].contiguous() if max_points is not None else out


def paired_batch(positions, n_pairs: int, sigma, gen, th_lim=(1e-3, math.pi - 1e-3)):
    """n_pairs base points drawn from positions [3, M] and partners displaced by
    N(0, sigma^2) per coordinate: device float64 [3, 2 n_pairs]."""
    import torch
    M = positions.shape[1]
    idx = torch.randint(0, M, (n_pairs,), device=positions.device, generator=gen)
    x = positions[:, idx]
    s = torch.as_tensor(sigma, dtype=torch.float64, device=positions.device)[:, None]
    xp = x + s * torch.randn(x.shape, dtype=torch.float64, device=positions.device, generator=gen)
    xp[1].clamp_(th_lim[0], th_lim[1])
    return torch.cat([x, xp], dim=1).contiguous()


def train(ctx, positions, steps: int, n_pairs: int, sigma, lr: float = 2e-3, lr_end: float = 2e-5,
          beta_pair: float = 10.0, wc=(1.0,) * 6, seed: int = 0, start_step: int = 1,
          log_every: int = 0) -> List[float]:
    """Adam with a cosine learning-rate schedule from lr to lr_end; targets are
    the grid's B and E at every point (gc_field_sample).  Returns the losses."""
    import torch
    gen = torch.Generator(device=positions.device)
    gen.manual_seed(seed)
    losses = []
    for i in range(steps):
        pts = paired_batch(positions, n_pairs, sigma, gen)
        tgt = ctx.field_sample(pts)[:, :6].contiguous()
        a = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * i / max(steps - 1, 1)))
        losses.append(ctx.mlp_train_step(pts, tgt, wc=wc, beta_pair=beta_pair, lr=a, step=start_step + i))
        if log_every and (i % log_every == 0 or i == steps - 1):
            print(f"  train step {i}: loss {losses[-1]:.4e} lr {a:.2e}", flush=True)
    return losses


def field_errors(ctx, pts) -> Dict[str, float]:
    """Error of the network against the grid at device points [3, n]: RMS over
    the points of |dB|/|B|, |dE|/|E|, |d grad|B|| / |grad|B|| and |dK|/|K| (K =
    (b.grad)b), each norm taken over the three components."""
    import torch
    g = ctx.field_sample(pts)
    m = ctx.mlp_eval(pts)
    out = {}
    for name, sl in (("B", slice(0, 3)), ("E", slice(3, 6)), ("G", slice(6, 9)), ("K", slice(9, 12))):
        num = torch.linalg.norm(m[:, sl] - g[:, sl], dim=1)
        den = torch.linalg.norm(g[:, sl], dim=1).clamp_min(1e-300)
        out[name] = float(torch.sqrt(torch.mean((num / den) ** 2)))
    return out
