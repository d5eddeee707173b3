"""Throughput of the guiding-centre push on one MI355X.

Workload (paper scale): 1,048,576 electrons at 81 keV injected at r = 0.28 AU,
24 deg latitude (longitude +-2 deg, pitch cosine uniform in [0, 1]), split in
three ensembles with mean free path 0.1, 0.5 and 1 AU; Parker spiral plus 16
seeded Fourier modes (dB/B = 0.1) on a 256x128x256 grid of 12 FP32 components
over [0.1, 2] AU; dt = 1 s; cell binning every 64 steps.

One bench step = one chunk of 64 guiding-centre steps of every active particle:
cell keys + radix sort + permute, the push kernel, and the snapshot moments.
The default --steps 1350 covers the full 24 h of simulated time.  The metric
counts steps of active particles only.

Prints one JSON line.  --gpus > 1 is rejected: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_STEP = {"f32": 768, "f64": 1536, "f16": 384}     # 2 gathers x 8 nodes x 12 components
PEAK_HBM_GBS = 8000.0
# VALU issue of MI355X: one wave64 instruction per 4 cycles per SIMD (16 lanes, full-rate FP64 FMA
# included), 256 CUs x 4 SIMDs at 2.4 GHz; in FP64 FMA flops this is the 78.6 TFLOP/s vector peak
PEAK_VALU_GINST = 256 * 4 * 2.4e9 / 4 / 1e9
PEAK_FP64_TFLOPS = 78.6
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "push_traffic.json")
VALU_JSON = os.path.join(ROOT, "profiles", "push_valu.json")
WHOLE_JOB_CHUNKS = 1350          # 24 h of 1 s steps in chunks of 64
KERNEL_SOURCES = ["paper_2403_06706_amd/csrc/gc_push.hip", "paper_2403_06706_amd/csrc/gc_step.h",
                  "paper_2403_06706_amd/csrc/gc_device.h", "paper_2403_06706_amd/csrc/gc_internal.h",
                  "paper_2403_06706_amd/csrc/gc_kernels.hip", "paper_2403_06706_amd/build.py"]


def kernel_hash() -> str:
    """Hash of the push and field-layout sources without their comments and
    blank lines (a change of wording does not invalidate measured counters)."""
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def moment_spec():
    from synthetic import AU, E_CHARGE

    class Spec:   # <sin^2 alpha>(r), energy vs age near 1 AU, pitch cosine of young electrons
        n_rbins, r_lo, r_hi = 38, 0.1 * AU, 2.0 * AU
        n_mubins, sel_r_lo, sel_r_hi = 36, 0.9 * AU, 1.1 * AU
        age_lo, age_hi, min_collisions = 0.0, 1200.0, 1
        n_agebins, age_max = 48, 48 * 3600.0
        n_ebins, e_lo, e_hi = 64, 70e3, 82e3
        e_unit, len_unit = E_CHARGE, AU
    return Spec


def build_workload(args):
    import numpy as np
    import torch
    from synthetic import workloads
    wl = workloads.config_paper_scale(seed=args.seed, n=args.particles, store_dtype=args.store)
    t0 = time.time()
    field = wl.build_field(wl.grid, device="cuda" if torch.cuda.is_available() else None)
    log(f"[bench] field {wl.grid.nr}x{wl.grid.nth}x{wl.grid.nph} built in {time.time() - t0:.1f} s")
    return wl, np.ascontiguousarray(field)


def hbm_copy_rate(ctx, n_bytes=2 << 30):
    """Achievable HBM bandwidth: gc_copy_probe over n_bytes (read + write bytes
    per second), timed with HIP events on the library's stream."""
    import torch
    src = torch.empty(n_bytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    ctx.copy_probe(dst, src, n_bytes)          # warm
    best = 0.0
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.copy_probe(dst, src, n_bytes)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        best = max(best, 2 * n_bytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    return best


def gather_ceiling(ctx, wl, store):
    """Gather-only probe (gc_gather_probe) and one push chunk from the same
    state (after the warmup), each timed with HIP events on the library's
    stream: the push as a fraction of the achievable gather rate."""
    import torch
    snap = {k: v.clone() for k, v in ctx.get_state().items()}
    out = {}
    for what in ("probe", "push"):
        ctx.set_state(snap)
        ctx.advance(wl.dt, 1)                    # reorder (live prefix, cell order) and one step
        torch.cuda.synchronize()
        ctx.reset_counters()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        if what == "probe":
            ctx.gather_probe(wl.dt, 64)
        else:
            ctx.advance(wl.dt, 64)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        c = ctx.counters()
        ms = e0.elapsed_time(e1) if what == "probe" else c["push_ms"]
        out[what] = {"particle_steps": c["particle_steps"], "ms": ms,
                     "rate": c["particle_steps"] / (ms * 1e-3)}
    ctx.set_state(snap)
    probe, push = out["probe"], out["push"]
    return {"kernel": "gc::k_gather_probe", "state": "after the warmup chunks, 64 steps",
            "hbm_copy_GBps": hbm_copy_rate(ctx),
            "gather_rate_particle_steps_per_s": probe["rate"],
            "gather_GBps": probe["rate"] * BYTES_PER_STEP[store] / 1e9,
            "push_rate_same_state": push["rate"], "push_frac_of_gather_ceiling": push["rate"] / probe["rate"]}


def run_gpu(args, wl, field, precision, steps, warmup, timing="push", probe=False, probe_ceiling=False, extra=None):
    import torch
    import paper_2403_06706_amd as gcp
    ctx = gcp.Context(device=0, precision=precision, order="bin", chunk_steps=64, block_size=args.block,
                      bin_coarsen=args.coarsen, persistent=args.persistent, tile=args.tile, timing=timing)
    ctx.load_field(wl.grid, field, args.store, extra=extra)
    for e in wl.ensembles:
        ctx.inject(e)
    start = {k: v.clone() for k, v in ctx.get_state().items()}
    spec = moment_spec()
    for _ in range(warmup):
        ctx.advance(wl.dt, 64)
        ctx.moments(spec)
    torch.cuda.synchronize()
    ceiling = gather_ceiling(ctx, wl, store=args.store) if (probe_ceiling and warmup > 0) else None
    ctx.set_state(start)                      # time the workload from injection
    ctx.reset_counters()
    if probe:   # traffic-counter calibration: a plain copy of known size before the push
        nbytes = 256 << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        ctx.copy_probe(dst, src, nbytes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mom = None
    for i in range(steps):
        ctx.advance(wl.dt, 64)
        mom = ctx.moments(spec)
        if (i + 1) % 200 == 0:
            log(f"[bench] {precision}: step {i + 1}/{steps}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    c = ctx.counters()
    final = gcp.state_to_numpy(ctx.get_state())
    m = mom.cpu().numpy() if mom is not None else None
    ctx.close()
    return elapsed, c, final, m, ceiling


def steady_spec(min_birth: int):
    from synthetic import AU, E_CHARGE

    class Spec:   # Sect. 3 steady-state statistics near 1 AU, electrons born after the steady state
        n_rbins, r_lo, r_hi = 38, 0.1 * AU, 2.0 * AU
        n_mubins, sel_r_lo, sel_r_hi = 36, 0.9 * AU, 1.1 * AU
        age_lo, age_hi, min_collisions = 0.0, 1e12, 0
        n_agebins, age_max = 96, 12 * 3600.0          # 7.5 min age bins
        n_ebins, e_lo, e_hi = 80, 62e3, 82e3          # 0.25 keV energy bins
        e_unit, len_unit = E_CHARGE, AU
    Spec.min_birth = min_birth
    return Spec


def run_steady(args, n=None, hours=None, field=None, with_cpu=True):
    """The steady-state run of Sect. 3 as one job: 10^3 electrons reborn at
    once whenever they leave the shell, 150 h of 0.54 s steps, <r>(t) after
    every 100 steps, and from 8.3 h on snapshots every 100 steps accumulated
    on the device, the binned sections keeping electrons born after 8.3 h."""
    import numpy as np
    import torch
    import paper_2403_06706_amd as gcp
    from synthetic import workloads, AU
    wl = workloads.config_steady(seed=args.seed, n=n or args.steady_particles,
                                 hours=hours or args.steady_hours, store_dtype=args.store)
    if getattr(args, "steady_wind", False):
        # Fig. 11 setting: centres moving with a 418 km/s wind, only v_par b kept
        from dataclasses import replace
        wl.ensembles = [replace(wl.ensembles[0], v_wind=418e3, drift_free=True)]
        wl.name += "-windframe"
    if field is None:
        field = np.ascontiguousarray(wl.build_field(wl.grid, device="cuda"))
    every = wl.bin_interval
    n_snap = wl.n_steps // every
    t_steady = 8.3 * 3600.0
    first = int(np.ceil(t_steady / wl.dt / every))          # first accumulated snapshot
    min_birth = int(np.ceil(t_steady / wl.dt))
    spec = steady_spec(min_birth)

    class Mean:   # <r> only: the eight scalar sums
        n_rbins = n_mubins = n_agebins = n_ebins = min_collisions = 0
        r_lo, r_hi, sel_r_lo, sel_r_hi, age_lo, age_hi, age_max = 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0
        e_lo, e_hi, e_unit, len_unit = 0.0, 1.0, 1.0, AU
    ctx = gcp.Context(device=0, precision=args.precision, order="bin", chunk_steps=every, timing=True)
    ctx.load_field(wl.grid, field, args.store)
    ctx.inject(wl.ensembles[0])
    acc = torch.zeros(ctx.moments_size(spec), dtype=torch.int64, device="cuda")
    series = torch.zeros((n_snap, 8), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(n_snap):
        ctx.advance(wl.dt, every)
        ctx.moments(Mean, out=series[j])
        if j + 1 >= first:
            ctx.moments(spec, out=acc, accumulate=True)
        if (j + 1) % 2000 == 0:
            log(f"[bench] steady: snapshot {j + 1}/{n_snap}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    c = ctx.counters()
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    ser = series.cpu().numpy()
    a = acc.cpu().numpy()
    r_mean = ser[:, 6] / 2.0 ** 32 / np.maximum(ser[:, 0], 1)          # AU
    t_h = (np.arange(n_snap) + 1) * every * wl.dt / 3600.0
    late = r_mean[len(r_mean) // 2:].mean()
    win = max(1, int(round(3600.0 / (every * wl.dt))))                   # one hour of snapshots
    smooth = np.convolve(r_mean, np.ones(win) / win, mode="valid")
    near = np.nonzero(np.abs(smooth - late) <= 0.02 * late)[0]
    nb = spec.n_rbins
    n_part = wl.ensembles[0].n
    gen = st["flags"].astype(np.uint32) >> np.uint32(8)
    out = {"workload": wl.name, "particles": n_part, "steps": wl.n_steps, "dt_s": wl.dt,
           "simulated_hours": wl.n_steps * wl.dt / 3600.0, "wall_s": round(elapsed, 3),
           "value": c["particle_steps"] / elapsed, "unit": "particle-steps/s",
           "snapshots_accumulated": int(n_snap - first + 1), "samples_accumulated": int(a[0]),
           "samples_per_electron_snapshot": a[0] / (n_part * (n_snap - first + 1)),
           "selected_binned_samples": int(a[8:8 + 3 * nb:3].sum()),
           "rebirths": int(gen.sum()), "rebirths_per_electron": float(gen.mean()),
           "r_mean_AU": {f"{h:g}h": round(float(r_mean[min(n_snap - 1, int(round(h * 3600 / wl.dt / every)) - 1)]), 4)
                         for h in (1, 2, 4, 8.3, 20, 50, 100, 150) if h * 3600 / wl.dt / every <= n_snap},
           "steady_after_h": round(float(t_h[near[0]]), 2) if len(near) else None,
           "energy_vs_age_near_1AU": energy_vs_age(a, spec),
           "forms": {"launches": c["form_launches"], "ms": [round(x, 1) for x in c["form_ms"]],
                     "particle_steps": c["form_steps"]}}
    log(f"[bench] steady: {out['value']:.3e} particle-steps/s, {elapsed:.1f} s for {out['simulated_hours']:.0f} h; "
        f"{out['rebirths_per_electron']:.1f} rebirths per electron; steady after {out['steady_after_h']} h")
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline_steady(args, wl, field)
    return out


def energy_vs_age(a, spec):
    """Mean kinetic energy (keV) of the accumulated electrons near 1 AU per age
    bin, and the loss rate (keV/h) at a few ages (central differences over
    +-2 bins), from the energy-vs-age histogram of the accumulated moments."""
    import numpy as np
    nb = spec.n_rbins
    h = a[8 + 3 * nb + spec.n_mubins:].reshape(spec.n_agebins, spec.n_ebins).astype(np.float64)
    e_mid = (spec.e_lo + (np.arange(spec.n_ebins) + 0.5) * (spec.e_hi - spec.e_lo) / spec.n_ebins) / 1e3
    cnt = h.sum(1)
    mean = np.where(cnt > 0, (h * e_mid).sum(1) / np.maximum(cnt, 1), np.nan)
    da = spec.age_max / spec.n_agebins / 3600.0
    age_mid = (np.arange(spec.n_agebins) + 0.5) * da
    def num(x):
        return None if not np.isfinite(x) else round(float(x), 3)
    out = {"samples": int(cnt.sum()),
           "mean_keV": {f"{t:g}h": num(mean[int(t / da)]) for t in (0.3, 0.5, 1, 2, 4, 8)}}
    rates = {}
    for t in (0.3, 1, 4):            # least-squares slope over the populated bins within +-2 of the age
        i = int(t / da)
        sel = [j for j in range(max(i - 2, 0), min(i + 3, spec.n_agebins)) if cnt[j] > 0]
        rates[f"{t:g}h"] = num(np.polyfit(age_mid[sel], mean[sel], 1)[0]) if len(sel) >= 2 else None
    out["loss_rate_keV_per_h"] = rates
    return out


def cpu_baseline_steady(args, wl, field):
    """The oracle on the same steady-state job, over a bounded share of its steps."""
    import numpy as np
    import oracle as O
    of = O.Field(wl.grid, field.astype(np.float32).astype(np.float64) if args.store == "f32" else field)
    tab = O.make_ens_table(wl.ensembles)
    p = O.inject(of, tab, 0, np.arange(wl.ensembles[0].n, dtype=np.uint32))
    steps = min(wl.n_steps, args.steady_cpu_steps)
    t0 = time.perf_counter()
    O.advance(of, tab, p, wl.dt, steps)
    el = time.perf_counter() - t0
    done = int(p["step"].astype(np.int64).sum())
    return {"value": done / el, "unit": "particle-steps/s", "cores": O.max_threads(), "kind": "oracle",
            "sample": f"{wl.ensembles[0].n} electrons x first {steps} steps of the run",
            "job_estimate_s": round(wl.n_steps / steps * el, 1)}


def run_batched(args, wl=None, field=None):
    """64 ensembles of uneven size (4M electrons), ragged stop times, advanced by
    the persistent push in hipGraph replays of 128 steps, launch parameters
    from the autotuner."""
    import numpy as np
    import torch
    import paper_2403_06706_amd as gcp
    from synthetic import workloads
    if wl is None:
        wl = workloads.config_batched(seed=args.seed, store_dtype=args.store)
        field = np.ascontiguousarray(wl.build_field(wl.grid, device="cuda"))
    stream = torch.cuda.Stream()
    ctx = gcp.Context(device=0, precision=args.precision, persistent=True, tile=args.tile, stream=stream)
    ctx.load_field(wl.grid, field, args.store)
    for e in wl.ensembles:
        ctx.inject(e)
    t0 = time.time()
    # the batched form is the persistent push: tune its workgroup, bin and tile sizes
    tune = ctx.autotune(wl.dt, probe_steps=128, blocks=(128, 256), coarsen=(0, 1), chunks=(),
                        tiles=(256, 512, 1024, 4096), cache=args.tune_cache, key=f"{wl.name}-{args.store}-{args.precision}")
    log(f"[bench] autotune ({time.time() - t0:.1f} s): {tune}")
    opts = {k: v for k, v in tune["options"].items() if k in ("block_size", "bin_coarsen", "tile", "chunk_steps")}
    ctx.close()
    ctx = gcp.Context(device=0, precision=args.precision, stream=stream, persistent=True, **opts)
    ctx.load_field(wl.grid, field, args.store)
    for e in wl.ensembles:
        ctx.inject(e)
    with torch.cuda.stream(stream):
        ctx.advance_graph(wl.dt, 128)              # capture and run once (warmup) ...
    stream.synchronize()
    ctx.close()
    ctx = gcp.Context(device=0, precision=args.precision, stream=stream, persistent=True, **opts)
    ctx.load_field(wl.grid, field, args.store)     # ... then time a fresh run from injection
    for e in wl.ensembles:
        ctx.inject(e)
    reps = (wl.n_steps + 127) // 128
    ctx.reset_counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for i in range(reps):
            ctx.advance_graph(wl.dt, 128)
            if (i + 1) % 300 == 0:
                log(f"[bench] batched: replay {i + 1}/{reps}")
    stream.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    c = ctx.counters()
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    value = c["particle_steps"] / el
    return {
        "metric": "GC particle-steps/s on 1 MI355X, batched ensembles (persistent push, hipGraph)",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": el / reps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "f64" else "f32", "data": "synthetic",
        "config": {"workload": wl.name, "particles": wl.n_particles, "ensembles": len(wl.ensembles),
                   "steps_per_bench_step": 128, "simulated_hours": reps * 128 * wl.dt / 3600.0,
                   "field_store": args.store, "form": "persistent", "tuned_options": opts,
                   "tune_rates": {"entry": tune["default_rate"], "best": tune["best_rate"], "tried": tune["n_tried"]}},
        "final_status_counts": np.bincount(st["status"], minlength=4).tolist(),
    }


# matrix-core work of one network evaluation: value + 3 tangent rows through
# 6 layers of 128 x 128 and the 128 -> 6 output layer, 2 flops per multiply-add
MLP_FLOPS_PER_EVAL = 4 * 2 * (6 * 128 * 128 + 6 * 128)
MLP_EVALS_PER_STEP = 2
PEAK_BF16_TFLOPS = 2500.0


def run_mlp(args, n_particles=None, steps=None, with_cpu=True):
    """Neural-field workload: electrons at 81 keV (lambda 0.5 AU) injected as in
    the small spiral workload, pushed through the network trained by the
    library on 49M positions drawn along trajectories of that workload (8,192
    electrons over 2 h on the 64x32x64 grid).  The grid stays loaded as fallback
    (cell binning) and as judge; the same particles are also timed through the
    grid for the speed-up."""
    import math
    from dataclasses import replace
    import numpy as np
    import torch
    import paper_2403_06706_amd as gcp
    from paper_2403_06706_amd import neural
    from synthetic import fields, workloads
    from synthetic.mlp_setup import init_params, make_spec
    small = workloads.config_small(n=8192)
    f = fields.parker(small.grid)
    t0 = time.time()
    tr = gcp.Context(device=0)
    tr.load_field(small.grid, f, "f64")
    tr.inject(small.ensembles[0])
    pos = neural.collect_positions(tr, small.dt, small.n_steps, every=16)
    spec = make_spec(small.grid, f, seed=1)
    tr.mlp_set(spec.freq, spec.r_ref, spec.scale, spec.power, init_params(seed=4))
    g = small.grid
    sigma = [0.1 * (g.r_max - g.r_min) / (g.nr - 1), 0.1 * math.pi / g.nth, 0.1 * 2 * math.pi / g.nph]
    torch.cuda.synchronize()
    t1 = time.time()
    losses = neural.train(tr, pos, steps=3000, n_pairs=8192, sigma=sigma, beta_pair=100.0, lr=2e-3, seed=0)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    held = gcp.Context(device=0)
    held.load_field(small.grid, f, "f64")
    held.inject(replace(small.ensembles[0], n=1024, seed=7))
    hold = neural.collect_positions(held, small.dt, small.n_steps, every=64)
    held.close()
    ferr = neural.field_errors(tr, hold)
    params = tr.mlp_params()
    tr.close()
    log(f"[bench] network trained in {t_train:.1f} s (set-up {t1 - t0:.1f} s), loss {losses[-1]:.3e}, "
        f"field error vs grid {ferr}")

    ens = replace(small.ensembles[0], n=n_particles or args.mlp_particles, seed=args.seed)
    if steps is None:
        steps = args.steps if args.steps is not None else 4

    def timed(source):
        ctx = gcp.Context(device=0, precision=args.precision, field_source=source, timing=True)
        ctx.load_field(small.grid, f, args.store)
        ctx.mlp_set(spec.freq, spec.r_ref, spec.scale, spec.power, params)
        ctx.inject(ens)
        start = {k: v.clone() for k, v in ctx.get_state().items()}
        for _ in range(args.warmup):
            ctx.advance(small.dt, 64)
        torch.cuda.synchronize()
        ctx.set_state(start)
        del start
        ctx.reset_counters()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            ctx.advance(small.dt, 64)
            log(f"[bench] {source}: chunk {i + 1}/{steps}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        c = ctx.counters()
        st = gcp.state_to_numpy(ctx.get_state())
        ctx.close()
        return el, c, st

    el, c, st = timed("mlp")
    value = c["particle_steps"] / el
    gel, gc_, gst = timed("grid")
    grid_value = gc_["particle_steps"] / gel
    avg = c["push_ms"] / 1e3 / max(c["n_push"], 1)
    per_launch = c["particle_steps"] / max(c["n_push"], 1)
    flops = MLP_FLOPS_PER_EVAL * MLP_EVALS_PER_STEP * per_launch
    achieved = flops / avg / 1e12
    # trajectory difference network vs grid over the window (same particles, same draws)
    both = (st["status"] == 0) & (gst["status"] == 0)
    R = lambda s: np.stack([s["r"] * np.sin(s["th"]) * np.cos(s["ph"]), s["r"] * np.sin(s["th"]) * np.sin(s["ph"]),
                            s["r"] * np.cos(s["th"])], 1)
    same_k = both & (st["k"] == gst["k"])
    d = np.linalg.norm(R(st)[same_k] - R(gst)[same_k], axis=1) / np.linalg.norm(R(gst)[same_k], axis=1)
    out = {
        "metric": "GC particle-steps/s on 1 MI355X, neural-field push",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": el / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"neural-field-spiral-{ens.n}", "particles": ens.n, "lambda_AU": ens.lambda_par / 1.495978707e11,
                   "ekin_keV": 81.0, "dt_s": small.dt, "steps_per_bench_step": 64,
                   "simulated_seconds": steps * 64 * small.dt, "state_precision": args.precision,
                   "network": "64 Fourier frequencies -> 6 x 128 SiLU -> 6, BF16 weights, FP32 accumulation",
                   "training": {"positions": int(pos.shape[1]), "samples": 3000 * 8192 * 2, "steps": 3000,
                                "seconds": round(t_train, 2), "final_loss": losses[-1]},
                   "field_error_vs_grid_rms": ferr},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "traffic": None, "kernel": "gc::k_push_mlp",
                     "avg_launch_ms": round(avg * 1e3, 3), "flops_per_particle_step": MLP_FLOPS_PER_EVAL * MLP_EVALS_PER_STEP,
                     "algorithmic_flops_per_launch": flops},
        "grid_push_same_particles": {"value": grid_value, "speedup_network_over_grid": value / grid_value},
        "trajectory_difference_vs_grid": {"particles": int(same_k.sum()), "median": float(np.median(d)) if len(d) else None,
                                          "max": float(d.max()) if len(d) else None},
    }
    if with_cpu and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_mlp(args, small, f, spec, params)
    return out


def cpu_baseline_mlp(args, small, f, spec, params):
    """The oracle integrator driven by the FP64 NumPy network, one point per
    call (as it stands, single-threaded), on a bounded sample of the workload."""
    from dataclasses import replace
    import numpy as np
    import oracle as O
    from oracle import mlp_oracle as M
    ens = replace(small.ensembles[0], n=96, seed=args.seed)
    tab = O.make_ens_table([ens])
    p = O.inject(O.Field(small.grid, f), tab, 0, np.arange(ens.n, dtype=np.uint32))
    pd = {k: np.asarray(v, dtype=np.float64) for k, v in params.items()}
    cb = O.Field(small.grid, callback=lambda r, th, ph: M.field(spec, pd, np.array([r]), np.array([th]), np.array([ph]))[0])
    t0 = time.perf_counter()
    O.advance(cb, tab, p, small.dt, 64, 1)
    el = time.perf_counter() - t0
    steps = int(p["step"].sum())
    return {"value": steps / el, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{ens.n} electrons x 64 steps through the FP64 NumPy network (one point per call); "
                      f"{steps} particle-steps in {el:.1f} s"}


def load_profile(path, args):
    """A committed counter summary of the push, if it belongs to these kernel
    sources, field store and precision (else None: the counters are stale)."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tj = json.load(f)
    if tj.get("kernel_hash") == kernel_hash() and tj.get("store") == args.store and tj.get("precision") == args.precision:
        return tj
    return None


# Counter passes over the push (one rocprofv3 --pmc run each, with the command
# PMC_BENCH_ARGS); their CSV output directories are named pmc_<pass>.
PMC_BENCH_ARGS = "--warmup 0 --no-cpu-baseline --probe-copy"
PMC_PASSES = {
    "p1": "SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_INSTS_VMEM_RD SQ_INSTS_SALU SQ_WAIT_INST_ANY "
          "SQ_BUSY_CYCLES SQ_WAVE_CYCLES GRBM_GUI_ACTIVE GRBM_COUNT",
    "p2": "SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_TRANS_F64 "
          "SQ_INSTS_VALU_CVT SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64 SQ_INSTS_VALU_FMA_F32 GRBM_GUI_ACTIVE",
    "p3": "TA_TA_BUSY_sum TA_FLAT_READ_WAVEFRONTS_sum TD_TD_BUSY_sum TD_TC_STALL_sum TCP_TOTAL_CACHE_ACCESSES_sum "
          "TCP_TCC_READ_REQ_sum TCP_PENDING_STALL_CYCLES_sum TCP_READ_TAGCONFLICT_STALL_CYCLES_sum GRBM_GUI_ACTIVE",
    "p5": "SQ_ACTIVE_INST_VMEM SQ_INST_CYCLES_VMEM_RD SQ_ACTIVE_INST_ANY SQ_THREAD_CYCLES_VALU SQ_WAIT_ANY "
          "SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VALU_FLOPS_FP64_TRANS SQ_CYCLES GRBM_GUI_ACTIVE",
    "t1": "FETCH_SIZE",
    "t2": "WRITE_SIZE",
    "t3": "TCC_HIT_sum TCC_MISS_sum",
}
PUSH_KERNEL = "k_push<0, 1, 0, true>"   # the tame-field instantiation (FP32 field of finite values)
COPY_KERNEL = "k_copy_probe"
N_CU = 256
N_XCD = 8          # GRBM_GUI_ACTIVE is summed over the XCDs
COPY_PROBE_KIB = 262144.0


def _pmc_dispatches(d, kernel):
    """Counters per dispatch of one kernel (dispatch order) from a rocprofv3 CSV."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    per = {}
    for fn in files:
        with open(fn) as f:
            for row in csv.DictReader(f):
                if kernel not in row["Kernel_Name"]:
                    continue
                c = per.setdefault(int(row["Dispatch_Id"]), {})
                c[row["Counter_Name"]] = c.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    return [per[k] for k in sorted(per)]


def _bench_line(path):
    with open(path) as f:
        lines = [ln for ln in f if ln.startswith('{"metric"')]
    if not lines:
        raise ValueError(f"no bench line in {path}")
    return json.loads(lines[-1])


def _launch_groups(n, max_rows=12, groups=10):
    """Row ranges [a, b) of the per-launch tables: every launch, or ten groups
    of consecutive launches when there are many."""
    if n <= max_rows:
        return [(i, i + 1) for i in range(n)]
    return [(n * g // groups, n * (g + 1) // groups) for g in range(groups)]


def _group_sums(launches, a, b):
    """Counter sums over launches [a, b) with their busy fractions."""
    g = {k: sum(x[k] for x in launches[a:b]) for k in launches[a]}
    cu_cycles = N_CU * g["GRBM_GUI_ACTIVE"] / N_XCD
    g["valu_busy"] = g["SQ_ACTIVE_INST_VALU"] / cu_cycles
    g["ta_busy"] = g["TA_TA_BUSY_sum"] / cu_cycles
    g["td_busy"] = g["TD_TD_BUSY_sum"] / cu_cycles
    g["label"] = f"{a + 1}" if b == a + 1 else f"{a + 1}–{b}"
    return g


def summarize_push_pmc(d, out_dir=None):
    """Writes push_valu.json, push_traffic.json and their tables (into
    profiles/, or out_dir) from the rocprofv3 passes PMC_PASSES under directory
    d (pmc_<pass>/ with the CSV output, pmc_<pass>.log with the bench line of
    that run).  Returns the two summaries."""
    launches, probe = None, {}
    lines = {}
    for name in PMC_PASSES:
        L = _pmc_dispatches(os.path.join(d, f"pmc_{name}"), PUSH_KERNEL)
        if launches is None:
            launches = [{"GRBM_GUI_ACTIVE": []} for _ in L]
        if len(L) != len(launches):
            raise ValueError(f"pass {name}: {len(L)} push launches, expected {len(launches)}")
        for acc, cs in zip(launches, L):
            for k, v in cs.items():
                if k == "GRBM_GUI_ACTIVE":
                    acc[k].append(v)
                else:
                    acc[k] = v
        for k, v in (_pmc_dispatches(os.path.join(d, f"pmc_{name}"), COPY_KERNEL) or [{}])[0].items():
            probe[k] = v
        lines[name] = _bench_line(os.path.join(d, f"pmc_{name}.log"))
    cfg = lines["p1"]["config"]
    rl = lines["p1"]["roofline"]
    if rl["launches"] != len(launches):
        raise ValueError("bench line and counters disagree on the number of push launches")
    steps = float(rl["particle_steps_per_launch"]) * rl["launches"]
    for acc in launches:
        acc["GRBM_GUI_ACTIVE"] = sum(acc["GRBM_GUI_ACTIVE"]) / len(acc["GRBM_GUI_ACTIVE"])
        cu_cycles = N_CU * acc["GRBM_GUI_ACTIVE"] / N_XCD
        acc["valu_busy"] = acc["SQ_ACTIVE_INST_VALU"] / cu_cycles   # quad-cycles per SIMD: 4 SIMDs per CU
        acc["ta_busy"] = acc["TA_TA_BUSY_sum"] / cu_cycles
        acc["td_busy"] = acc["TD_TD_BUSY_sum"] / cu_cycles
    tot = {k: sum(a[k] for a in launches) for k in launches[0]}
    cu_cycles = N_CU * tot["GRBM_GUI_ACTIVE"] / N_XCD
    pps = {k: v / steps for k, v in tot.items() if k.startswith(("SQ_", "TA_", "TD_", "TCP_", "TCC_"))}
    h = kernel_hash()
    kname = f"gc::{PUSH_KERNEL} (FP64 arithmetic, FP32 field, plain mode, throughput form)"
    cmd = f"bench.py {PMC_BENCH_ARGS}"
    valu = {
        "kernel": kname, "kernel_hash": h, "store": cfg["field_store"], "precision": cfg["precision"],
        "launches": len(launches), "particle_steps": steps, "per_particle_step": pps,
        "valu_instructions_per_particle_step": pps["SQ_INSTS_VALU"],
        "fp64_flops_per_particle_step": 64.0 * pps["SQ_INSTS_VALU_FLOPS_FP64"],
        "valu_busy": tot["SQ_ACTIVE_INST_VALU"] / cu_cycles,
        "ta_busy": tot["TA_TA_BUSY_sum"] / cu_cycles, "td_busy": tot["TD_TD_BUSY_sum"] / cu_cycles,
        "l1_tag_accesses_per_load": tot["TCP_TOTAL_CACHE_ACCESSES_sum"] / tot["TA_FLAT_READ_WAVEFRONTS_sum"],
        "derivation": f"sums over the {len(launches)} launches of gc::{PUSH_KERNEL} in '{cmd}' ({steps:.5g} active "
                      f"particle-steps), one rocprofv3 --pmc pass per counter set; busy fractions = counter / "
                      f"({N_CU} CUs x GRBM_GUI_ACTIVE / {N_XCD} XCDs); written by bench.py --summarize-push-pmc"}
    fetch_scale = COPY_PROBE_KIB / probe["FETCH_SIZE"]
    write_scale = COPY_PROBE_KIB / probe["WRITE_SIZE"]
    fetch_total, write_total = tot["FETCH_SIZE"] * fetch_scale, tot["WRITE_SIZE"] * write_scale
    hbm = 1024.0 * (fetch_total + write_total)
    traffic = {
        "kernel": kname, "kernel_hash": h, "store": cfg["field_store"], "precision": cfg["precision"],
        "hbm_bytes_per_particle_step": hbm / steps,
        "l2_hit_rate": tot["TCC_HIT_sum"] / (tot["TCC_HIT_sum"] + tot["TCC_MISS_sum"]),
        "l2_requests_per_particle_step": (tot["TCC_HIT_sum"] + tot["TCC_MISS_sum"]) / steps,
        "fetch_scale": fetch_scale, "write_scale": write_scale,
        "derivation": f"FETCH_SIZE x {fetch_scale:.4f} + WRITE_SIZE x {write_scale:.4f} (KiB; scales from the "
                      f"{COPY_PROBE_KIB:.0f} KiB copy of gc_copy_probe in the same runs) over {steps:.5g} "
                      f"particle-steps of '{cmd}'; written by bench.py --summarize-push-pmc"}
    prof = out_dir or os.path.join(ROOT, "profiles")
    valu_json = os.path.join(prof, os.path.basename(VALU_JSON))
    traffic_json = os.path.join(prof, os.path.basename(TRAFFIC_JSON))
    with open(valu_json, "w") as f:
        json.dump(valu, f, indent=1)
    with open(traffic_json, "w") as f:
        json.dump(traffic, f, indent=1)
    pmc_cmds = "\n".join(
        f"    rocprofv3 --pmc {PMC_PASSES[n]} \\\n        --kernel-include-regex 'k_push<|k_copy_probe' "
        f"--output-format csv -d $D/pmc_{n} -o run -- python3 $R/{cmd} > $D/pmc_{n}.log" for n in PMC_PASSES)
    head = (f"Commands (one counter set per run, no other tracing; run from `/tmp` with `TMPDIR=/tmp`, `$R` = "
            f"repository root, `$D` = an output directory), then `python3 $R/bench.py --summarize-push-pmc $D`, "
            f"which wrote this file's tables and `{os.path.basename(VALU_JSON)}` / "
            f"`{os.path.basename(TRAFFIC_JSON)}` (kernel source hash `{h}`):\n\n{pmc_cmds}\n\n"
            f"Workload: the paper-scale job (2^20 electrons, 256x128x256 FP32 field, chunks of 64 steps) as the "
            f"bench line times it; the counters cover its {len(launches)} launches of the throughput form, "
            f"{steps:.5g} active particle-steps (`roofline.particle_steps_per_launch` x `roofline.launches` of the "
            f"bench line), the tail forms are not counted.  `--probe-copy` first runs `gc_copy_probe`, a 256 MiB "
            f"copy, and skips every sub-record.\n")
    groups = [_group_sums(launches, a, b) for a, b in _launch_groups(len(launches))]
    rows = "\n".join(
        f"| {a['label']} | {a['SQ_INSTS_VALU']:,.0f} | {a['SQ_ACTIVE_INST_VALU']:,.0f} | {a['GRBM_GUI_ACTIVE']:,.0f} | "
        f"{a['valu_busy']:.3f} | {a['TA_TA_BUSY_sum']:,.0f} | {a['ta_busy']:.3f} | {a['td_busy']:.3f} | "
        f"{a['SQ_INSTS_VALU_CVT']:,.0f} | {a['SQ_INSTS_VALU_FLOPS_FP64']:,.0f} |" for a in groups)
    mix = [("FMA F64", "SQ_INSTS_VALU_FMA_F64"), ("MUL F64", "SQ_INSTS_VALU_MUL_F64"),
           ("ADD F64", "SQ_INSTS_VALU_ADD_F64"), ("transcendental F64", "SQ_INSTS_VALU_TRANS_F64"),
           ("conversions", "SQ_INSTS_VALU_CVT"), ("INT32", "SQ_INSTS_VALU_INT32"), ("INT64", "SQ_INSTS_VALU_INT64")]
    iv = pps["SQ_INSTS_VALU"]
    other = iv - sum(pps[k] for _, k in mix)
    mixrows = "\n".join(f"| {n} | {pps[k]:.3f} | {100 * pps[k] / iv:.1f} % |" for n, k in mix)
    with open(os.path.join(prof, "push_f64_f32field_paper_scale_valu.md"), "w") as f:
        f.write(f"""# k_push (FP64 arithmetic, FP32 field), paper-scale workload — VALU and vector-memory counters

What limits the throughput form of the grid push, `gc::{PUSH_KERNEL}`, on the paper-scale workload: its
vector ALU (VALU) issue is busy {valu['valu_busy']:.1%} of the cycles the SIMDs have, the texture-address (TA)
and texture-data (TD) paths of the field gathers {valu['ta_busy']:.1%} and {valu['td_busy']:.1%}; the HBM traffic
is {traffic['hbm_bytes_per_particle_step']:.1f} B per particle-step, {traffic['hbm_bytes_per_particle_step'] * steps / len(launches) / 1e9:.2f} GB per launch
(`push_f64_f32field_paper_scale_traffic.md`).

{head}
`GRBM_GUI_ACTIVE` is summed over the {N_XCD} XCDs ({N_XCD} x the kernel's cycles), averaged over the passes;
busy fractions are counter / ({N_CU} CUs x GRBM_GUI_ACTIVE / {N_XCD}).  `SQ_ACTIVE_INST_VALU` counts VALU
quad-cycles per SIMD, so it divides by {N_CU} CUs for 4 SIMDs.

Per launch (or, for many launches, summed over groups of consecutive launches):

| Launches | SQ_INSTS_VALU | SQ_ACTIVE_INST_VALU | GRBM_GUI_ACTIVE | VALU busy | TA_TA_BUSY_sum | TA busy | TD busy | SQ_INSTS_VALU_CVT | SQ_INSTS_VALU_FLOPS_FP64 |
|---|---|---|---|---|---|---|---|---|---|
{rows}

Sums over the {len(launches)} launches, per active particle-step (wavefront instructions; one wavefront
instruction serves up to 64 particles):

| VALU instructions | per particle-step | share |
|---|---|---|
{mixrows}
| other (moves, selects, compares, bit operations) | {other:.3f} | {100 * other / iv:.1f} % |
| **all VALU** | **{iv:.3f}** | 100 % |

* **VALU issue: {iv:.2f} wavefront instructions per particle-step**, busy {valu['valu_busy']:.3f} of the SIMD
  cycles.  The VALU issue peak of MI355X is one wave64 instruction per 4 cycles per SIMD (16 lanes;
  full-rate FP64 FMA included): 256 CUs x 4 SIMDs x 2.4 GHz / 4 = 614.4 G instructions/s, the 78.6 TFLOP/s
  FP64 vector peak counted in instructions.  bench.py reports `roofline.achieved` = {iv:.3f} x
  (particle-steps per launch) / (mean launch time from HIP events) against that peak.
* FP64 arithmetic: {valu['fp64_flops_per_particle_step']:.0f} FLOP per particle-step
  (`SQ_INSTS_VALU_FLOPS_FP64` x 64 lanes), of which 384 are the 2 x 96 interpolation FMAs.
* Vector memory: TA busy {valu['ta_busy']:.3f}, TD busy {valu['td_busy']:.3f};
  {valu['l1_tag_accesses_per_load']:.1f} L1 tag accesses per 16-byte-per-lane load (16 for 64 lanes on
  consecutive addresses); {pps['TCP_TCC_READ_REQ_sum']:.4f} L2 read requests per particle-step.
* {pps['SQ_INSTS_VALU_CVT']:.2f} conversions per particle-step are the FP32 field values widened to FP64
  (96 per gather).
""")
    trows = "\n".join(
        f"| {a['label']} | {a['FETCH_SIZE']:,.1f} | {a['WRITE_SIZE']:,.1f} | {a['TCC_HIT_sum']:,.0f} | {a['TCC_MISS_sum']:,.0f} | "
        f"{a['TCC_HIT_sum'] / (a['TCC_HIT_sum'] + a['TCC_MISS_sum']):.3f} |" for a in groups)
    with open(os.path.join(prof, "push_f64_f32field_paper_scale_traffic.md"), "w") as f:
        f.write(f"""# k_push (FP64 arithmetic, FP32 field), paper-scale workload — HBM and L2 counters

{head}
Calibration (same runs):

| Kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) |
|---|---|---|
| `gc::{COPY_KERNEL}` (256 MiB copy) | {probe['FETCH_SIZE']:,.1f} | {probe['WRITE_SIZE']:,.1f} |

so FETCH_SIZE is scaled by {COPY_PROBE_KIB:,.0f} / {probe['FETCH_SIZE']:,.1f} = {fetch_scale:.3f} and WRITE_SIZE by
{write_scale:.3f}.

Push launches (`gc::{PUSH_KERNEL}`; for many launches, sums over groups of consecutive launches):

| Launches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | TCC_HIT | TCC_MISS | L2 hit rate |
|---|---|---|---|---|---|
{trows}

* Scaled HBM bytes: {hbm:.4e} B over {steps:.5g} particle-steps = **{hbm / steps:.2f} B per active particle-step**,
  against 768 B per step of algorithmic field gathers (2 gathers x 8 nodes x 12 FP32 components): the
  gathers are served by the caches, and the HBM traffic is the particle state, written once per 64-step
  launch in slot order and read once through the last reorder's permutation, whose scattered 8-byte loads
  fetch whole cache lines: {fetch_total / max(write_total, 1.0):.1f} times the bytes written are fetched.
* L2: {traffic['l2_requests_per_particle_step']:.4f} requests per particle-step, hit rate {traffic['l2_hit_rate']:.3f}.
""")
    print(json.dumps({"valu": valu_json, "traffic": traffic_json, "kernel_hash": h,
                      "valu_instructions_per_particle_step": iv, "valu_busy": valu["valu_busy"],
                      "hbm_bytes_per_particle_step": traffic["hbm_bytes_per_particle_step"]}))
    return valu, traffic


def push_roofline(args, c):
    """Roofline of the dominant kernel, the throughput form of the push
    (gc::k_push): bound by its VALU issue (profiles/push_valu.json).  achieved =
    VALU wavefront instructions per active particle-step (committed counters)
    x particle-steps per launch / mean launch time (HIP events of this run)."""
    n0 = max(c["form_launches"][0], 1)
    avg_push_s = c["form_ms"][0] / 1e3 / n0
    steps_per_launch = c["form_steps"][0] / n0
    valu = load_profile(VALU_JSON, args)
    tj = load_profile(TRAFFIC_JSON, args)
    traffic = round(tj["hbm_bytes_per_particle_step"] * steps_per_launch) if tj else None
    gather_gbps = BYTES_PER_STEP[args.store] * steps_per_launch / avg_push_s / 1e9
    tail = {}
    for i, name in ((1, "gc::k_push_allpairs"), (2, "gc::k_push_quad")):
        if c["form_launches"][i]:
            tail[name] = {"launches": c["form_launches"][i], "avg_launch_ms": c["form_ms"][i] / c["form_launches"][i],
                          "particle_steps": c["form_steps"][i],
                          "rate": c["form_steps"][i] / (c["form_ms"][i] * 1e-3) if c["form_ms"][i] else None}
    r = {"bound": "alu", "unit": "Ginst/s", "peak": PEAK_VALU_GINST, "achieved": None, "frac": None,
         "traffic": traffic, "kernel": "gc::k_push", "avg_launch_ms": round(avg_push_s * 1e3, 4),
         "launches": c["form_launches"][0], "particle_steps_per_launch": round(steps_per_launch),
         "peak_derivation": "VALU issue: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction",
         "counters": "profiles/push_valu.json" if valu else "stale or missing (kernel sources changed)"}
    if valu:
        ipt = valu["valu_instructions_per_particle_step"]
        achieved = ipt * steps_per_launch / avg_push_s / 1e9
        flops = valu["fp64_flops_per_particle_step"] * steps_per_launch / avg_push_s / 1e12
        r.update({"achieved": round(achieved, 1), "frac": round(achieved / PEAK_VALU_GINST, 4),
                  "valu_instructions_per_particle_step": round(ipt, 3),
                  "valu_busy_in_profile": round(valu["valu_busy"], 3),
                  "fp64": {"flops_per_particle_step": round(valu["fp64_flops_per_particle_step"], 1),
                           "TFLOPs": round(flops, 2), "frac_of_78.6": round(flops / PEAK_FP64_TFLOPS, 4)},
                  "vector_memory_in_profile": {"ta_busy": round(valu["ta_busy"], 3), "td_busy": round(valu["td_busy"], 3),
                                               "l1_tag_accesses_per_load": round(valu["l1_tag_accesses_per_load"], 2)}})
    r["gathers"] = {"algorithmic_bytes_per_particle_step": BYTES_PER_STEP[args.store],
                    "logical_GBps": round(gather_gbps, 1), "served_by": "L1/L2 (HBM traffic in 'traffic')"}
    if tj:
        r["hbm_l2_from_counters"] = {
            "hbm_GBps": round(traffic / avg_push_s / 1e9, 1), "hbm_frac_of_peak": round(traffic / avg_push_s / 1e9 / PEAK_HBM_GBS, 4),
            "l2_hit_rate": tj.get("l2_hit_rate"), "l2_requests_per_particle_step": tj.get("l2_requests_per_particle_step"),
            "source": "profiles/push_traffic.json (rocprofv3 FETCH_SIZE, WRITE_SIZE, TCC_HIT, TCC_MISS)"}
    r["tail_forms"] = tail
    return r


def whole_job(args, wl, field):
    """The whole 24 h paper-scale job from injection (1,350 chunks of 64 steps,
    with the tail forms once few electrons remain), timed like the main run."""
    el, c, final, mom, _ = run_gpu(args, wl, field, args.precision, WHOLE_JOB_CHUNKS, 1, timing=True)
    total_ms = el * 1e3
    return {"chunks": WHOLE_JOB_CHUNKS, "simulated_hours": WHOLE_JOB_CHUNKS * 64 * wl.dt / 3600.0,
            "value": c["particle_steps"] / el, "particle_steps": c["particle_steps"], "wall_s": round(el, 3),
            "push_ms": round(c["push_ms"], 1), "reorder_ms": round(c["reorder_ms"], 1),
            "reorder_share": round(c["reorder_ms"] / total_ms, 4),
            "forms": {"launches": c["form_launches"], "ms": [round(x, 1) for x in c["form_ms"]],
                      "particle_steps": c["form_steps"]},
            "active_at_end": int((final["status"] == 0).sum())}


def precision_forms_gpu(args):
    """The small spiral workload (1,024 electrons, 2 h, lambda 0.5 AU) in every
    arithmetic and field-storage form on the device, with collision logs and
    |B| at the final positions sampled by the device; compared with the FP64
    oracle in the CPU-baseline leg."""
    import numpy as np
    import torch
    import paper_2403_06706_amd as gcp
    from synthetic import workloads
    wl = workloads.config_small()
    f64 = wl.build_field(wl.grid)
    f32 = f64.astype(np.float32).astype(np.float64)
    out = []
    for prec, store in (("f64", "f32"), ("f32_acc64", "f32"), ("f32_kahan", "f32"), ("f32_kahan", "f16"),
                        ("f64", "f16")):
        ctx = gcp.Context(device=0, precision=prec, log_depth=256)
        ctx.load_field(wl.grid, f32 if store == "f32" else f64, store)
        ctx.inject(wl.ensembles[0])
        ctx.advance(wl.dt, wl.n_steps)
        st = gcp.state_to_numpy(ctx.get_state())
        log = ctx.get_log().cpu().numpy().view(np.uint32)
        pts = torch.tensor(np.stack([st["r"], st["th"], st["ph"]]), dtype=torch.float64, device="cuda").contiguous()
        bmag = np.linalg.norm(ctx.field_sample(pts).cpu().numpy()[:, 0:3], axis=1)
        ctx.close()
        out.append({"precision": prec, "fields": store, "state": st, "log": log, "bmag": bmag})
    return wl, f32, out


def run_batched_pair(args):
    """The 64-ensemble workload (4M electrons, ragged stops up to 48 h) twice
    from injection: the graph-replayed persistent form with autotuned sizes,
    and the eager grid form (gc_advance, default sizes, tail policy)."""
    import numpy as np
    import torch
    import paper_2403_06706_amd as gcp
    from synthetic import workloads
    wl = workloads.config_batched(seed=args.seed, store_dtype=args.store)
    field = np.ascontiguousarray(wl.build_field(wl.grid, device="cuda"))
    graph = run_batched(args, wl=wl, field=field)
    ctx = gcp.Context(device=0, precision=args.precision)       # untimed, as the graph replays
    ctx.load_field(wl.grid, field, args.store)
    for e in wl.ensembles:
        ctx.inject(e)
    reps = (wl.n_steps + 127) // 128
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(reps):
        ctx.advance(wl.dt, 128)
        if (i + 1) % 300 == 0:
            log(f"[bench] batched eager: {i + 1}/{reps}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    c = ctx.counters()
    st = gcp.state_to_numpy(ctx.get_state())
    ctx.close()
    eager = {"value": c["particle_steps"] / el, "wall_s": round(el, 3), "particle_steps": c["particle_steps"],
             "form": "eager grid form (gc_advance, 64-thread workgroups, tail policy)",
             "final_status_counts": np.bincount(st["status"], minlength=4).tolist()}
    return {"workload": graph["config"]["workload"], "particles": graph["config"]["particles"],
            "ensembles": graph["config"]["ensembles"], "simulated_hours": graph["config"]["simulated_hours"],
            "graph_persistent": {"value": graph["value"], "wall_s": round(graph["ms_per_step"] * graph["steps"] / 1e3, 3),
                                 "tuned_options": graph["config"]["tuned_options"],
                                 "tune_rates": graph["config"]["tune_rates"],
                                 "final_status_counts": graph["final_status_counts"]},
            "eager": eager, "ratio_graph_persistent_over_eager": graph["value"] / eager["value"]}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def precision_table(forms):
    """CPU-baseline leg: the FP64 oracle on the small workload (FP32-rounded
    field, collision logs), timed, and each device form's final positions,
    energies and decisions against it.  Particles whose status, step, collision
    count and collision log agree with the oracle's are compared; the others
    are counted (decisions taken one step apart by round-off)."""
    import numpy as np
    import oracle as O
    from synthetic import C_LIGHT, E_CHARGE, M_ELECTRON
    wl, f32, runs = forms
    of = O.Field(wl.grid, f32)
    tab = O.make_ens_table(wl.ensembles)
    p = O.inject(of, tab, 0, np.arange(wl.ensembles[0].n, dtype=np.uint32))
    t0 = time.perf_counter()
    logs = O.advance(of, tab, p, wl.dt, wl.n_steps, O.max_threads(), log_depth=256)
    el = time.perf_counter() - t0
    olog = logs[0]
    b_o = np.array([np.linalg.norm(O.field_eval(of, p["r"][i], p["th"][i], p["ph"][i])[0][0:3]) for i in range(len(p))])

    def energy_ev(B, u, mu):
        return (np.sqrt(1 + (u ** 2 + 2 * mu * B) / C_LIGHT ** 2) - 1) * M_ELECTRON * C_LIGHT ** 2 / E_CHARGE

    e_o = energy_ev(b_o, p["u"], p["mu_B"] / M_ELECTRON)
    R = lambda r, th, ph: np.stack([r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)], 1)
    rows = []
    for run in runs:
        st, glog = run["state"], run["log"]
        same = ((st["k"] == p["k"]) & (st["step"] == p["step"]) & (st["status"] == p["status"])
                & np.all(glog == olog, axis=1))
        Rg, Ro = R(st["r"], st["th"], st["ph"])[same], R(p["r"], p["th"], p["ph"])[same]
        pos = np.linalg.norm(Rg - Ro, axis=1) / np.linalg.norm(Ro, axis=1)
        e_g = energy_ev(run["bmag"], st["u"], st["mu"])[same]
        de = np.abs(e_g - e_o[same]) / e_o[same]
        rows.append({"precision": run["precision"], "fields": run["fields"], "agreeing": int(same.sum()),
                     "decisions_differing": int((~same).sum()),
                     "rel_position": {"max": float(pos.max()), "median": float(np.median(pos))},
                     "rel_energy": {"max": float(de.max()), "median": float(np.median(de))}})
    return {"workload": f"spiral-64x32x64-{wl.ensembles[0].n}e-2h", "particles": int(len(p)), "steps": wl.n_steps,
            "reference": "FP64 oracle on the FP32-rounded field", "bar_fp64": 1e-6, "bar_fp32": 1e-4, "forms": rows,
            "oracle": {"value": int(p["step"].astype(np.int64).sum()) / el, "unit": "particle-steps/s",
                       "cores": O.max_threads(), "seconds": round(el, 3)}}


def cpu_baseline(args, wl, field):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np
    import oracle as O
    n_per = args.cpu_particles // len(wl.ensembles)
    of = O.Field(wl.grid, field.astype(np.float32).astype(np.float64) if args.store == "f32" else field)
    tab = O.make_ens_table(wl.ensembles)
    p = np.concatenate([O.inject(of, tab, i, np.arange(n_per, dtype=np.uint32))
                        for i, e in enumerate(wl.ensembles)])
    threads = O.max_threads()
    t0 = time.perf_counter()
    O.advance(of, tab, p, wl.dt, args.cpu_steps, threads)
    el = time.perf_counter() - t0
    steps = int(p["step"].sum())
    return {"value": steps / el, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(p)} electrons (ids 0..{n_per - 1} of each ensemble) x {args.cpu_steps} steps "
                      f"of the same field and injection; {steps} active particle-steps in {el:.1f} s",
            "cpu_model": cpu_model(), "per_core": steps / el / threads}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="chunks of 64 steps (default: 1350 = 24 h for the paper workload, 4 for the network)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--particles", type=int, default=1 << 20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--store", default="f32", choices=["f32", "f64", "f16"])
    ap.add_argument("--precision", default="f64", choices=["f64", "f32_acc64", "f32_kahan"])
    ap.add_argument("--block", type=int, default=64)
    ap.add_argument("--coarsen", type=int, default=0)
    ap.add_argument("--persistent", action="store_true")
    ap.add_argument("--tile", type=int, default=1024)
    ap.add_argument("--forms", type=int, default=None,
                    help="time the FP32 forms over this many chunks (default: the whole run; 0: skip)")
    ap.add_argument("--no-neural", action="store_true", help="skip the neural-field summary of the default run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-particles", type=int, default=98304)
    ap.add_argument("--cpu-steps", type=int, default=14400)
    ap.add_argument("--probe-copy", action="store_true", help="run a 256 MiB copy kernel first (counter calibration)")
    ap.add_argument("--workload", default="paper", choices=["paper", "batched", "mlp", "steady"])
    ap.add_argument("--steady-particles", type=int, default=1000)
    ap.add_argument("--steady-hours", type=float, default=150.0)
    ap.add_argument("--steady-cpu-steps", type=int, default=20000)
    ap.add_argument("--no-steady", action="store_true", help="skip the steady-state summary of the default run")
    ap.add_argument("--full-chunks", type=int, default=200,
                    help="chunks of the paper-scale job timed with the full Eqs. 1-2 (0: skip)")
    ap.add_argument("--steady-wind", action="store_true",
                    help="steady-state job with scattering in the wind frame and only v_par b (Fig. 11 setting)")
    ap.add_argument("--mlp-particles", type=int, default=10 << 20)
    ap.add_argument("--tune-cache", default=None, help="autotuner JSON cache (batched workload)")
    ap.add_argument("--no-whole-job", action="store_true", help="skip the whole-24 h sub-record")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched graph-versus-eager sub-record")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision-form table")
    ap.add_argument("--summarize-push-pmc", metavar="DIR", default=None,
                    help="write the push counter summaries under profiles/ from rocprofv3 passes in DIR (no GPU)")
    args = ap.parse_args()
    if args.summarize_push_pmc:
        summarize_push_pmc(args.summarize_push_pmc)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the guiding-centre push is data-parallel over particles "
              "and the library has no multi-GPU path (particles would be sharded by id, the field replicated, "
              "and the integer moments summed by one all-reduce).", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "batched":
        print(json.dumps(run_batched_pair(args)), flush=True)
        return
    if args.workload == "mlp":
        print(json.dumps(run_mlp(args)), flush=True)
        return
    if args.workload == "steady":
        print(json.dumps(run_steady(args)), flush=True)
        return
    if args.steps is None:
        args.steps = 1350
    wl, field = build_workload(args)
    log(f"[bench] {wl.n_particles} electrons, {len(wl.ensembles)} ensembles; warmup {args.warmup}, "
        f"timed {args.steps} chunks of 64 steps")
    elapsed, c, final, mom, ceiling = run_gpu(args, wl, field, args.precision, args.steps, args.warmup,
                                              probe=args.probe_copy, probe_ceiling=not args.probe_copy)
    value = c["particle_steps"] / elapsed
    log(f"[bench] {c['particle_steps']:.3e} particle-steps in {elapsed:.2f} s -> {value:.3e}/s; "
        f"push {c['push_ms']:.0f} ms over {c['n_push']} launches")

    roofline = push_roofline(args, c)
    roofline["gather_ceiling"] = ceiling
    out = {
        "metric": "GC particle-steps/s on 1 MI355X at <=1e-4 rel err vs FP64 oracle",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "f64" else "f32", "data": "synthetic",
        "config": {"workload": wl.name, "particles": wl.n_particles, "ensembles_lambda_AU": [0.1, 0.5, 1.0],
                   "ekin_keV": 81.0, "dt_s": wl.dt, "steps_per_bench_step": 64,
                   "simulated_hours": args.steps * 64 * wl.dt / 3600.0, "field_store": args.store,
                   "precision": args.precision, "order": "bin", "block": args.block,
                   "persistent": args.persistent},
        "roofline": roofline,
        "active_at_end": int((final["status"] == 0).sum()),
        "moments_last": {"active": int(mom[0]), "exited": int(mom[1]), "collisions": int(mom[4])} if mom is not None else None,
    }

    forms_steps = args.steps if args.forms is None else args.forms
    if forms_steps > 0 and not args.probe_copy:
        # the FP32 forms over the same job, as speed-ups over the plain push (their error
        # against the FP64 oracle is bounded by the precision tests)
        forms = {}
        for prec in ("f32_acc64", "f32_kahan"):
            if prec == args.precision:
                continue
            el, cc, _, _, _ = run_gpu(args, wl, field, prec, forms_steps, 1)
            v = cc["particle_steps"] / el
            forms[prec] = {"value": v, "speedup": v / value if forms_steps == args.steps else None}
            log(f"[bench] form {prec}: {v:.3e} particle-steps/s")
        out["forms"] = {"chunks": forms_steps, **forms}

    if not args.no_neural and not args.probe_copy:
        log("[bench] neural-field summary ...")
        nf = run_mlp(args, n_particles=2 << 20, steps=2, with_cpu=False)
        out["neural_field"] = {"value": nf["value"], "particles": nf["config"]["particles"],
                               "chunks": nf["steps"], "roofline": nf["roofline"],
                               "grid_push_same_particles": nf["grid_push_same_particles"],
                               "field_error_vs_grid_rms": nf["config"]["field_error_vs_grid_rms"],
                               "trajectory_difference_vs_grid": nf["trajectory_difference_vs_grid"],
                               "note": "full measurement: bench.py --workload mlp"}

    if args.full_chunks > 0 and not args.probe_copy:
        # the full Eqs. 1-2 (terms with derivatives of b and v_E) against the reduced form,
        # over the first chunks of the same job
        import numpy as np
        from synthetic import fields
        log("[bench] full-equation summary ...")
        t0 = time.time()
        extra = np.ascontiguousarray(fields.perturbed_parker_extra(wl.grid, device="cuda"))
        log(f"[bench] extra node array built in {time.time() - t0:.1f} s")
        el_f, cf, fin_f, _, _ = run_gpu(args, wl, field, args.precision, args.full_chunks, 1, extra=extra)
        el_r, cr, fin_r, _, _ = run_gpu(args, wl, field, args.precision, args.full_chunks, 1)
        act = (fin_f["status"] == 0) & (fin_r["status"] == 0)
        dr = np.abs(fin_f["r"] - fin_r["r"])[act] / 1.495978707e11
        out["full_equations"] = {
            "chunks": args.full_chunks, "value": cf["particle_steps"] / el_f,
            "reduced_same_chunks": cr["particle_steps"] / el_r,
            "ratio": (cf["particle_steps"] / el_f) / (cr["particle_steps"] / el_r),
            "r_difference_AU": {"median": float(np.median(dr)), "max": float(dr.max())} if act.any() else None}
        log(f"[bench] full equations: {out['full_equations']['value']:.3e} particle-steps/s "
            f"({out['full_equations']['ratio']:.2f} of the reduced form)")

    if not args.no_steady and not args.probe_copy:
        log("[bench] steady-state summary ...")
        out["steady_state"] = run_steady(args, field=field, with_cpu=False)
        out["steady_state"]["note"] = "with the oracle beside it: bench.py --workload steady"
        if not args.steady_wind:
            # the same job with scattering in the wind frame and only v_par b (Fig. 11 setting)
            wind_args = argparse.Namespace(**vars(args))
            wind_args.steady_wind = True
            log("[bench] steady-state summary, wind-frame scattering ...")
            out["steady_state_wind"] = run_steady(wind_args, field=field, with_cpu=False)
            out["steady_state_wind"]["note"] = "with the oracle beside it: bench.py --workload steady --steady-wind"

    if args.steps < WHOLE_JOB_CHUNKS and not args.no_whole_job and not args.probe_copy:
        log("[bench] whole 24 h job ...")
        out["whole_job"] = whole_job(args, wl, field)
        log(f"[bench] whole job: {out['whole_job']['value']:.3e} particle-steps/s in {out['whole_job']['wall_s']} s")

    if not args.no_batched and not args.probe_copy:
        log("[bench] batched 64-ensemble workload: graph + persistent against eager ...")
        out["batched"] = run_batched_pair(args)
        log(f"[bench] batched: graph+persistent {out['batched']['graph_persistent']['value']:.3e}, "
            f"eager {out['batched']['eager']['value']:.3e} particle-steps/s")

    forms_gpu = None
    if not args.no_precision and not args.probe_copy and not args.no_cpu_baseline:
        log("[bench] precision forms on the small workload ...")
        forms_gpu = precision_forms_gpu(args)

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(args, wl, field)
        log(f"[bench] oracle {out['cpu_baseline']['value']:.3e} particle-steps/s on {out['cpu_baseline']['cores']} threads")
        if forms_gpu is not None:
            out["precision_forms"] = precision_table(forms_gpu)
            for row in out["precision_forms"]["forms"]:
                log(f"[bench] form {row['precision']}/{row['fields']}: max rel position {row['rel_position']['max']:.2e}, "
                    f"{row['decisions_differing']} decisions differ")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
