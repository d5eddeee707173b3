"""Reduced-precision forms against the FP64 oracle.

Forms: FP32 field interpolation and right-hand side with FP64 position/u/time
accumulators; FP32 throughout with Kahan-compensated accumulation; the latter
with FP16 field storage (per-component power-of-two scales).

The oracle runs on its own (FP64) and logs its collision steps; so does the
device.  Round-off can move a collision (or an exit) by a step, a decision
taken in floating point.  Particles whose decisions agree are compared to the
1e-4 bar (relative position over 2 h); a particle whose decisions differ must
have been marginal: at the first differing decision the oracle's own free-path
margin |s - l| / l (or its distance to the exit shell) is within the reach of
FP32 round-off.  The FP16-field forms move the field itself; their errors are
reported, not bounded.
"""
import json
import os

import numpy as np
import pytest
from scipy import stats

import oracle as O
from gpu_helpers import (device_bmag, field_of, oracle_bmag, stored, run_gpu, run_oracle, rel_errors, small,
                         say)
from synthetic import M_ELECTRON, C_LIGHT, E_CHARGE

pytestmark = pytest.mark.gpu
DEPTH = 256
FLIP_MARGIN = 1e-4        # relative: free-path or exit-shell margin a FP32 run may decide the other way
NONE = 0xFFFFFFFF
OUT = os.environ.get("GC_REPORT_DIR")   # optional: directory for the per-form error reports (JSON)


def _energy_ev(B, u, mu):
    p2 = u ** 2 + 2 * mu * B
    gam = np.sqrt(1 + p2 / C_LIGHT ** 2)
    return (gam - 1) * M_ELECTRON * C_LIGHT ** 2 / E_CHARGE


def _oracle_margin(wl, of, tab, i, window):
    """Smallest decision margin of the oracle's own particle i over the steps
    start < n <= end of window: after each step, |s - l| / l (the collision
    test) and the relative distance to the exit shell (the exit test).  A flip
    between the FP32 device run and the FP64 oracle is legitimate when such a
    near-tie lies between the last decision both sides share and the oracle's
    side of the first decision that differs."""
    start, end = window
    e = wl.ensembles[0]
    q = O.inject(of, tab, 0, np.array([i], dtype=np.uint32))
    if start:
        O.advance(of, tab, q, wl.dt, start, 1)
    best = np.inf
    for _ in range(end - start):
        if q["status"][0] != O.ACTIVE:
            break
        O.advance(of, tab, q, wl.dt, 1, 1)
        if np.isfinite(q["ell"][0]):
            best = min(best, abs(q["s"][0] - q["ell"][0]) / q["ell"][0])
        r = q["r"][0]
        best = min(best, abs(r - e.r_in) / e.r_in, abs(r - e.r_out) / e.r_out)
    return best


def _oracle_window(i, glog, p, olog):
    """Oracle step counts (start, end] that hold the first decision on which the
    two runs differ: from the last collision both logged alike to the oracle's
    next collision (or its last step)."""
    diff = np.nonzero(glog[i] != olog[i])[0]
    d = int(diff[0]) if len(diff) else int(np.sum(olog[i] != NONE))
    start = int(olog[i][d - 1]) if d > 0 else 0
    end = int(olog[i][d]) if len(diff) and olog[i][d] != NONE else int(p["step"][i])
    return start, max(end, start)


@pytest.mark.parametrize("prec,store,tol", [("f32_acc64", "f32", 1e-4), ("f32_kahan", "f32", 1e-4),
                                            ("f32_kahan", "f16", None), ("f64", "f16", None)])
def test_form_error_against_fp64_oracle(prec, store, tol):
    wl = small()                                  # 1,024 electrons, 2 h, lambda = 0.5 AU
    f64 = field_of(wl)
    f_ref = stored(f64, "f32")                    # FP64 state with FP32 fields is the reference
    say(f"precision form {prec} / fields {store}")
    st, glog = run_gpu(wl, f_ref if store == "f32" else f64, store_dtype=store, precision=prec, log_depth=DEPTH)
    p, logs, of, tab = run_oracle(wl, f_ref, log_depth=DEPTH)
    olog = logs[0]
    assert int(np.sum(st["k"] > DEPTH)) == 0 and int(np.sum(p["k"] > DEPTH)) == 0
    same = ((st["k"] == p["k"]) & (st["step"] == p["step"]) & (st["status"] == p["status"])
            & np.all(glog == olog, axis=1))
    flipped = np.nonzero(~same)[0]
    sub = {k: v[same] for k, v in st.items()}
    pos, u, mu = rel_errors(sub, p[same], M_ELECTRON)
    b_gpu = device_bmag(wl, f_ref if store == "f32" else f64, store, sub["r"], sub["th"], sub["ph"])
    e_gpu = _energy_ev(b_gpu, sub["u"], sub["mu"])
    b_ora = oracle_bmag(of, p["r"][same], p["th"][same], p["ph"][same])
    e_ora = _energy_ev(b_ora, p["u"][same], p["mu_B"][same] / M_ELECTRON)
    de = np.abs(e_gpu - e_ora)
    report = {"form": prec, "fields": store, "particles": int(len(st["r"])), "steps": wl.n_steps,
              "agreeing": int(same.sum()), "flips": int(len(flipped)), "max_rel_pos": float(pos.max()),
              "median_rel_pos": float(np.median(pos)), "max_rel_u": float(u.max()), "max_rel_mu": float(mu.max()),
              "max_abs_energy_eV": float(de.max()), "median_abs_energy_eV": float(np.median(de))}
    say("  " + json.dumps(report))
    if OUT:
        os.makedirs(OUT, exist_ok=True)
        with open(os.path.join(OUT, f"precision_{prec}_{store}.json"), "w") as fh:
            json.dump(report, fh)
    if tol is not None:
        assert pos.max() <= tol, report
        assert u.max() <= tol and mu.max() <= tol, report
        assert len(flipped) <= 0.01 * len(st["r"]), report
        for i in flipped:
            m = _oracle_margin(wl, of, tab, i, _oracle_window(i, glog, p, olog))
            assert m <= FLIP_MARGIN, (int(i), m)


@pytest.mark.parametrize("prec", ["f32_kahan"])
def test_long_run_statistics_match(prec):
    """6 h of 4,096 electrons: the distributions of final pitch cosine, radius and
    energy-loss rate of the FP32 form agree with the FP64 oracle (KS p > 0.01)."""
    wl = small(n=4096, hours=6.0)
    f = stored(field_of(wl), "f32")
    st, _ = run_gpu(wl, f, store_dtype="f32", precision=prec)
    p, *_ = run_oracle(wl, f)
    of = O.Field(wl.grid, f)
    a_g = st["status"] == 0
    a_o = p["status"] == 0
    assert abs(int(a_g.sum()) - int(a_o.sum())) <= max(10, 0.01 * len(p))
    b_g = device_bmag(wl, f, "f32", st["r"][a_g], st["th"][a_g], st["ph"][a_g])
    b_o = oracle_bmag(of, p["r"][a_o], p["th"][a_o], p["ph"][a_o])
    mu_g = st["u"][a_g] / np.sqrt(st["u"][a_g] ** 2 + 2 * st["mu"][a_g] * b_g)
    mu_o = p["u"][a_o] / np.sqrt(p["u"][a_o] ** 2 + 2 * (p["mu_B"][a_o] / M_ELECTRON) * b_o)
    assert stats.ks_2samp(mu_g, mu_o).pvalue > 0.01
    assert stats.ks_2samp(st["r"][a_g], p["r"][a_o]).pvalue > 0.01
    e0 = 81e3
    rate_g = (_energy_ev(b_g, st["u"][a_g], st["mu"][a_g]) - e0) / st["t"][a_g]
    rate_o = (_energy_ev(b_o, p["u"][a_o], p["mu_B"][a_o] / M_ELECTRON) - e0) / p["t"][a_o]
    assert stats.ks_2samp(rate_g, rate_o).pvalue > 0.01
    assert abs(rate_g.mean() - rate_o.mean()) <= 0.01 * abs(rate_o.mean()) + 3 * rate_o.std() / np.sqrt(len(rate_o))
