"""Shared helpers of the GPU tests: run a workload through the C ABI and
through the oracle, and compare per particle."""
import math
import sys
from dataclasses import replace

import numpy as np

import oracle as O
from synthetic import workloads

_FIELD_CACHE = {}


def field_of(wl, device=None):
    key = (wl.name, wl.grid)
    if key not in _FIELD_CACHE:
        _FIELD_CACHE[key] = wl.build_field(wl.grid, device=device) if device else wl.build_field(wl.grid)
    return _FIELD_CACHE[key]


def stored(field, store_dtype):
    """The values the device holds, as float64 (the oracle reads the same numbers)."""
    if store_dtype == "f32":
        return field.astype(np.float32).astype(np.float64)
    return field


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(wl, field, store_dtype="f64", precision="f64", order="bin", chunk=64, n_steps=None, dt=None,
            log_depth=0, block=None, persistent=False, tile=1024, coarsen=0, ensembles=None, graph=False,
            tail_threshold=None, extra=None):
    import torch
    import paper_2403_06706_amd as gcp
    stream = torch.cuda.Stream() if graph else None
    if graph and tail_threshold is None:
        tail_threshold = 0          # pure replays (with a threshold, the tail runs eagerly)
    ctx = gcp.Context(device=0, precision=precision, order=order, chunk_steps=chunk, log_depth=log_depth,
                      block_size=block, persistent=persistent, tile=tile, bin_coarsen=coarsen, stream=stream,
                      tail_threshold=tail_threshold)
    ctx.load_field(wl.grid, field, store_dtype, extra=extra)
    for e in (ensembles or wl.ensembles):
        ctx.inject(e)
    n = wl.n_steps if n_steps is None else n_steps
    if n:
        if graph:
            with torch.cuda.stream(stream):
                ctx.advance_graph(wl.dt if dt is None else dt, n)
        else:
            ctx.advance(wl.dt if dt is None else dt, n)
    st = gcp.state_to_numpy(ctx.get_state())
    log = ctx.get_log().cpu().numpy().view(np.uint32) if log_depth else None
    ctx.close()
    return st, log


def run_oracle(wl, field, n_steps=None, dt=None, ensembles=None, ids=None, log_depth=0, threads=0, extra=None):
    ens = ensembles or wl.ensembles
    of = O.Field(wl.grid, field, extra=extra)
    tab = O.make_ens_table(ens)
    parts = []
    for i, e in enumerate(ens):
        sel = np.arange(e.n, dtype=np.uint32) if ids is None else np.asarray(ids[i], dtype=np.uint32)
        parts.append(O.inject(of, tab, i, sel))
    p = np.concatenate(parts) if parts else np.zeros(0, dtype=O.PARTICLE_DTYPE)
    n = wl.n_steps if n_steps is None else n_steps
    logs = O.advance(of, tab, p, wl.dt if dt is None else dt, n, threads, log_depth=log_depth)
    return p, logs, of, tab


def cart(r, th, ph):
    return np.stack([r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)], axis=-1)


def rel_errors(st, p, m):
    """Per-particle relative errors of position (Cartesian, |dR|/|R|), of u and of
    mu = mu_B/m (each relative to its largest value in the ensemble)."""
    Rg = cart(st["r"], st["th"], st["ph"])
    Ro = cart(p["r"], p["th"], p["ph"])
    pos = np.linalg.norm(Rg - Ro, axis=1) / np.linalg.norm(Ro, axis=1)
    u = np.abs(st["u"] - p["u"]) / max(np.abs(p["u"]).max(), 1.0)     # relative to the largest |p|/m
    mu_o = p["mu_B"] / m
    mu = np.abs(st["mu"] - mu_o) / np.maximum(np.abs(mu_o).max(), 1e-300)
    return pos, u, mu


def compare(st, p, m, tol, what=""):
    """Same status, step and collision count for every particle; position, u and
    mu within tol.  Returns the error arrays."""
    assert len(st["r"]) == len(p), (len(st["r"]), len(p))
    flips = np.nonzero((st["status"] != p["status"]) | (st["k"] != p["k"]) | (st["step"] != p["step"]))[0]
    assert len(flips) == 0, f"{what}: {len(flips)} particles differ in status/step/collisions, first {flips[:5]}"
    pos, u, mu = rel_errors(st, p, m)
    assert pos.max() <= tol, f"{what}: max relative position error {pos.max():.3e} > {tol}"
    assert u.max() <= tol, f"{what}: max relative u error {u.max():.3e} > {tol}"
    assert mu.max() <= tol, f"{what}: max relative mu error {mu.max():.3e} > {tol}"
    return pos, u, mu


def oracle_to_state(p, m):
    """Oracle particles as a device state (gc_set_state layout: mu = mu_B / m,
    zero compensation terms)."""
    import torch
    d = {"r": p["r"], "th": p["th"], "ph": p["ph"], "u": p["u"], "mu": p["mu_B"] / m,
         "fr": p["fp"][:, 0], "fth": p["fp"][:, 1], "fph": p["fp"][:, 2], "fu": p["fp"][:, 3],
         "dtp": p["dtp"], "s": p["s"], "ell": p["ell"], "t": p["t"]}
    for k in ("cr", "cth", "cph", "cu", "ct"):
        d[k] = np.zeros(len(p))
    out = {k: torch.tensor(np.ascontiguousarray(v, dtype=np.float64)) for k, v in d.items()}
    u32 = {k: p[k] for k in ("k", "status", "step", "id", "ens", "birth")}
    u32["flags"] = p["flags"] | (p["gen"] << np.uint32(GEN_SHIFT))
    for k, v in u32.items():
        out[k] = torch.tensor(np.ascontiguousarray(v, dtype=np.uint32).view(np.int32))
    return out


GEN_SHIFT = 8     # device flags: generation in the bits from here up


def state_to_oracle(st, m):
    """A device state (state_to_numpy of gc_get_state, injection order) as
    oracle particles (the inverse of oracle_to_state)."""
    p = np.zeros(len(st["r"]), dtype=O.PARTICLE_DTYPE)
    for k in ("r", "th", "ph", "u", "dtp", "s", "ell", "t"):
        p[k] = st[k]
    p["mu_B"] = st["mu"] * m
    p["fp"] = np.stack([st["fr"], st["fth"], st["fph"], st["fu"]], axis=1)
    for k in ("k", "status", "step", "id", "ens", "birth"):
        p[k] = st[k]
    flags = st["flags"].astype(np.uint32)
    p["flags"] = flags & np.uint32((1 << GEN_SHIFT) - 1)
    p["gen"] = flags >> np.uint32(GEN_SHIFT)
    return p


def generation(st):
    return st["flags"].astype(np.uint32) >> np.uint32(GEN_SHIFT)


def device_bmag(wl, field, store_dtype, r, th, ph):
    """|B| at points by the device's own trilinear sampling of the loaded grid
    (derived quantities of device results come from the device side)."""
    import torch
    import paper_2403_06706_amd as gcp
    if len(r) == 0:
        return np.zeros(0)
    ctx = gcp.Context(device=0)
    ctx.load_field(wl.grid, field, store_dtype)
    pts = torch.tensor(np.stack([r, th, ph]), dtype=torch.float64, device="cuda:0").contiguous()
    g = ctx.field_sample(pts).cpu().numpy()
    ctx.close()
    return np.linalg.norm(g[:, 0:3], axis=1)


def oracle_bmag(of, r, th, ph):
    out = np.full(len(r), np.nan)
    for i in range(len(r)):
        g, ok = O.field_eval(of, r[i], th[i], ph[i])
        if ok:
            out[i] = np.linalg.norm(g[0:3])
    return out


def small(n=1024, hours=2.0, **kw):
    wl = workloads.config_small(n=n, hours=hours)
    if kw:
        wl.ensembles = [replace(wl.ensembles[0], **kw)]
    return wl


def same_state(a, b, keys=None):
    keys = keys or [k for k in a if k not in ("cr", "cth", "cph", "cu", "ct")]
    for k in keys:
        if not np.array_equal(a[k], b[k], equal_nan=True):
            bad = np.nonzero(~((a[k] == b[k]) | (np.isnan(a[k]) & np.isnan(b[k])) if a[k].dtype.kind == "f"
                               else a[k] != b[k]))[0]
            raise AssertionError(f"state '{k}' differs at {len(bad)} particles, first {bad[:5]}")


del math
