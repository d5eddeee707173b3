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
from gpu_helpers import field_of, stored, run_gpu, run_oracle, rel_errors, small, say
from synthetic import M_ELECTRON, C_LIGHT, E_CHARGE

pytestmark = pytest.mark.gpu
DEPTH = 256
FLIP_MARGIN = 1e-4        # relative: free-path or exit-shell margin a FP32 run may decide the other way
NONE = 0xFFFFFFFF
OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")


def _energy_ev(field, r, th, ph, u, mu):
    out = np.zeros(len(r))
    for i in range(len(r)):
        g, ok = O.field_eval(field, r[i], th[i], ph[i])
        B = np.linalg.norm(g[0:3]) if ok else np.nan
        p2 = u[i] ** 2 + 2 * mu[i] * B
        gam = np.sqrt(1 + p2 / C_LIGHT ** 2)
        out[i] = (gam - 1) * M_ELECTRON * C_LIGHT ** 2 / E_CHARGE
    return out


def _decision_margin(wl, of, tab, i, st, glog, p, olog):
    """Oracle margin at the first decision on which device and oracle differ
    for particle i: |s - l| / l after the step whose end decided a collision,
    else the relative distance to the exit shell after the earlier exit."""
    e = wl.ensembles[0]
    diff = np.nonzero(glog[i] != olog[i])[0]
    q = O.inject(of, tab, 0, e, np.array([i], dtype=np.uint32))
    if len(diff):
        d = diff[0]
        n0 = int(min(glog[i][d], olog[i][d]))
        O.advance(of, tab, q, wl.dt, n0, 1)
        return abs(q["s"][0] - q["ell"][0]) / q["ell"][0]
    n0 = int(min(st["step"][i], p["step"][i]))
    O.advance(of, tab, q, wl.dt, n0 - 1, 1)        # the last step both sides took
    r = q["r"][0]
    return min(abs(r - e.r_in) / e.r_in, abs(r - e.r_out) / e.r_out)


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
    e_gpu = _energy_ev(of, sub["r"], sub["th"], sub["ph"], sub["u"], sub["mu"])
    e_ora = _energy_ev(of, p["r"][same], p["th"][same], p["ph"][same], p["u"][same], p["mu_B"][same] / M_ELECTRON)
    de = np.abs(e_gpu - e_ora)
    report = {"form": prec, "fields": store, "particles": int(len(st["r"])), "steps": wl.n_steps,
              "agreeing": int(same.sum()), "flips": int(len(flipped)), "max_rel_pos": float(pos.max()),
              "median_rel_pos": float(np.median(pos)), "max_rel_u": float(u.max()), "max_rel_mu": float(mu.max()),
              "max_abs_energy_eV": float(de.max()), "median_abs_energy_eV": float(np.median(de))}
    say("  " + json.dumps(report))
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, f"precision_{prec}_{store}.json"), "w") as fh:
        json.dump(report, fh)
    if tol is not None:
        assert pos.max() <= tol, report
        assert u.max() <= tol and mu.max() <= tol, report
        assert len(flipped) <= 0.01 * len(st["r"]), report
        for i in flipped:
            m = _decision_margin(wl, of, tab, i, st, glog, p, olog)
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
    def pitch(r, th, ph, u, mu):
        out = np.zeros(len(r))
        for i in range(len(r)):
            g, _ = O.field_eval(of, r[i], th[i], ph[i])
            out[i] = u[i] / np.sqrt(u[i] ** 2 + 2 * mu[i] * np.linalg.norm(g[0:3]))
        return out
    mu_g = pitch(st["r"][a_g], st["th"][a_g], st["ph"][a_g], st["u"][a_g], st["mu"][a_g])
    mu_o = pitch(p["r"][a_o], p["th"][a_o], p["ph"][a_o], p["u"][a_o], p["mu_B"][a_o] / M_ELECTRON)
    assert stats.ks_2samp(mu_g, mu_o).pvalue > 0.01
    assert stats.ks_2samp(st["r"][a_g], p["r"][a_o]).pvalue > 0.01
    e0 = 81e3
    rate_g = (_energy_ev(of, st["r"][a_g], st["th"][a_g], st["ph"][a_g], st["u"][a_g], st["mu"][a_g]) - e0) / st["t"][a_g]
    rate_o = (_energy_ev(of, p["r"][a_o], p["th"][a_o], p["ph"][a_o], p["u"][a_o], p["mu_B"][a_o] / M_ELECTRON) - e0) / p["t"][a_o]
    assert stats.ks_2samp(rate_g, rate_o).pvalue > 0.01
    assert abs(rate_g.mean() - rate_o.mean()) <= 0.01 * abs(rate_o.mean()) + 3 * rate_o.std() / np.sqrt(len(rate_o))
