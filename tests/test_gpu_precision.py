"""Reduced-precision forms against the FP64 oracle.

Forms: FP32 field interpolation and right-hand side with FP64 position/u/time
accumulators; FP32 throughout with Kahan-compensated accumulation; the latter
with FP16 field storage (per-component power-of-two scales).

Round-off can move a collision (or an exit) by a step.  Each device run logs
its collision steps; the oracle then replays the same collision schedule and
step count, and the trajectories are compared at identical times.  Bar: 1e-4
relative position error over 2 h for the FP32 forms with FP32 fields (the
spec tolerance); the FP16-field form is reported, not bounded.
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


@pytest.mark.parametrize("prec,store,tol", [("f32_acc64", "f32", 1e-4), ("f32_kahan", "f32", 1e-4),
                                            ("f32_kahan", "f16", None), ("f64", "f16", None)])
def test_form_error_against_fp64_oracle(prec, store, tol):
    wl = small()                                  # 1,024 electrons, 2 h, lambda = 0.5 AU
    f64 = field_of(wl)
    f_ref = stored(f64, "f32")                    # FP64 state with FP32 fields is the reference
    say(f"precision form {prec} / fields {store}")
    st, log = run_gpu(wl, f_ref if store == "f32" else f64, store_dtype=store, precision=prec, log_depth=DEPTH)
    normal, *_ = run_oracle(wl, f_ref)
    flips = int(np.sum((st["k"] != normal["k"]) | (st["step"] != normal["step"]) | (st["status"] != normal["status"])))
    over = int(np.sum(st["k"] > DEPTH))
    of = O.Field(wl.grid, f_ref)
    tab = O.make_ens_table(wl.ensembles)
    rep = O.inject(of, tab, 0, wl.ensembles[0], np.arange(wl.ensembles[0].n, dtype=np.uint32))
    O.advance_replay(of, tab, rep, wl.dt, st["step"], log)
    ok = st["k"] <= DEPTH
    sub = {k: v[ok] for k, v in st.items()}
    pos, u, mu = rel_errors(sub, rep[ok], M_ELECTRON)
    e_gpu = _energy_ev(of, sub["r"], sub["th"], sub["ph"], sub["u"], sub["mu"])
    e_ora = _energy_ev(of, rep["r"][ok], rep["th"][ok], rep["ph"][ok], rep["u"][ok], rep["mu_B"][ok] / M_ELECTRON)
    de = np.abs(e_gpu - e_ora)
    report = {"form": prec, "fields": store, "particles": int(len(st["r"])), "steps": wl.n_steps,
              "flips": flips, "beyond_log": over, "max_rel_pos": float(pos.max()), "median_rel_pos": float(np.median(pos)),
              "max_rel_u": float(u.max()), "max_rel_mu": float(mu.max()), "max_abs_energy_eV": float(de.max()),
              "median_abs_energy_eV": float(np.median(de))}
    say("  " + json.dumps(report))
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, f"precision_{prec}_{store}.json"), "w") as fh:
        json.dump(report, fh)
    assert over == 0
    # replayed trajectories use the device's collision schedule: same collision count
    assert np.array_equal(rep["k"][ok], sub["k"])
    if tol is not None:
        assert pos.max() <= tol, report
        assert u.max() <= tol and mu.max() <= tol, report


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
