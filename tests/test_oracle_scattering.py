"""Pins of the oracle's hard-sphere scattering (Eqs. 9, 10, 12): free-path and
isotropy statistics, exact collision scheduling in a uniform field, and the
equivalence of the exponential free path with the paper's per-step draw."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from synthetic import AU, SphericalGrid, fields, C_LIGHT, M_ELECTRON
from synthetic.constants import KEV
from synthetic.workloads import Ensemble

G = SphericalGrid(16, 8, 8, 0.1 * AU, 2.0 * AU)
STRAIGHT = fields.straight(G)


def _run(n=2000, lam=0.02 * AU, steps=400, law=0, mode=0, seed=0, depth=64, mu_lo=-1.0, mu_hi=1.0):
    field = O.Field(G, STRAIGHT)
    e = Ensemble(n=n, ensemble=2, seed=seed, r0=1.0 * AU, lat0=0.0, dlon=0.5, lambda_par=lam,
                 r_in=0.11 * AU, r_out=1.85 * AU, scatter_law=law, mu_lo=mu_lo, mu_hi=mu_hi)
    tab = O.make_ens_table([e], collision_mode=mode)
    p = O.inject(field, tab, 0, np.arange(n, dtype=np.uint32))
    ell0 = p["ell"].copy()
    u0 = p["u"].copy()
    logs = O.advance(field, tab, p, 1.0, steps, log_depth=depth)
    return p, logs, ell0, u0, e


def test_free_paths_are_exponential_with_mean_lambda():
    lam = 0.02 * AU
    p, (steps, mu, ell), ell0, _, _ = _run(lam=lam)
    ells = np.concatenate([ell0, ell[np.isfinite(ell)]]) / lam
    assert len(ells) > 10000
    assert stats.kstest(ells, "expon").pvalue > 0.01
    assert abs(ells.mean() - 1.0) < 3.0 / math.sqrt(len(ells))


def test_post_collision_pitch_cosine_isotropic():
    """Eq. 10: mu' = 1 - 2a is uniform on (-1, 1], so <mu'^2> = 1/3 and
    <sin^2 alpha> = 2/3 (the isotropic value quoted with Fig. 3)."""
    p, (steps, mu, ell), *_ = _run()
    m = mu[np.isfinite(mu)]
    assert len(m) > 10000
    assert stats.kstest(m, stats.uniform(loc=-1, scale=2).cdf).pvalue > 0.01
    s2 = 1 - m * m
    assert abs(s2.mean() - 2.0 / 3.0) < 3 * s2.std() / math.sqrt(len(s2))


def test_flux_weighted_law_eq12():
    """Eq. 12: mu' = +-sqrt(a): |mu'| has CDF x^2, both signs equally likely."""
    p, (steps, mu, ell), *_ = _run(law=1)
    m = mu[np.isfinite(mu)]
    assert stats.kstest(np.abs(m), lambda x: np.clip(x, 0, 1) ** 2).pvalue > 0.01
    frac_pos = (m > 0).mean()
    assert abs(frac_pos - 0.5) < 3 * 0.5 / math.sqrt(len(m))


def test_collision_scheduling_is_exact_in_uniform_field():
    """In a uniform field |v_par| is constant between collisions, so the path
    per step is |v_par| dt and collision k+1 is applied at the start of the
    step after the one where the path reaches ell_k: the gap in steps is
    ceil(ell_k / (|v_par| dt))."""
    p, (steps, mu, ell), ell0, u0, e = _run(n=400, steps=600)
    gam = 1.0 + e.ekin / (M_ELECTRON * C_LIGHT ** 2)
    v = C_LIGHT * math.sqrt(1 - 1 / gam ** 2)
    checked = 0
    for i in range(len(p)):
        prev_step, prev_ell, prev_vpar = 0, ell0[i], abs(u0[i]) / gam
        for k in range(steps.shape[1]):
            if steps[i, k] == 0xFFFFFFFF:
                break
            ratio = prev_ell / (prev_vpar * 1.0)
            frac = ratio - math.floor(ratio)
            if 1e-9 < frac < 1 - 1e-9:
                assert steps[i, k] - prev_step == math.ceil(ratio)
                checked += 1
            prev_step, prev_ell, prev_vpar = steps[i, k], ell[i, k], abs(mu[i, k]) * v
    assert checked > 2000


def test_exponential_free_path_matches_per_step_draw_of_eq9():
    """READING check: drawing exp(lambda) free paths per collision index is
    equivalent in distribution to the paper's per-step collision test
    a < 1 - exp(-ds/lambda) (memorylessness).  Compare collision counts."""
    n, steps = 6000, 150
    pa, *_ = _run(n=n, steps=steps, mode=0, depth=0, mu_lo=0.2, mu_hi=1.0)
    pb, *_ = _run(n=n, steps=steps, mode=1, depth=0, mu_lo=0.2, mu_hi=1.0)
    ka = pa["k"].astype(float)
    kb = pb["k"].astype(float)
    assert ka.mean() > 1.0
    se = math.sqrt(ka.var() / n + kb.var() / n)
    assert abs(ka.mean() - kb.mean()) < 4 * se
    assert stats.ks_2samp(ka, kb).pvalue > 0.001


def test_energy_and_position_kept_at_collision():
    """Inertial-frame scattering (Sect. 3): |p| unchanged, so gamma is unchanged."""
    p, (steps, mu, ell), _, u0, e = _run(n=200, steps=300)
    m = e.m
    Bmag = STRAIGHT[0, 0, 0, 0]
    p2_end = (m * p["u"]) ** 2 + 2 * m * p["mu_B"] * Bmag
    gam = 1.0 + e.ekin / (m * C_LIGHT ** 2)
    p2_0 = (m * C_LIGHT) ** 2 * (gam ** 2 - 1)
    assert np.allclose(p2_end, p2_0, rtol=1e-13)
    assert (p["k"] > 0).mean() > 0.5


def test_paper_collision_time_scale():
    """Sect. 3: 100 steps of 0.54 s (54 s) are about a tenth of the collision
    time at lambda = 0.5 AU for 81 keV electrons; the injected speed gives
    lambda/v close to 500 s."""
    field = O.Field(G, STRAIGHT)
    e = Ensemble(n=1, ensemble=0, seed=0, r0=1.0 * AU, lat0=0.0, mu_lo=1.0, mu_hi=1.0,
                 lambda_par=0.5 * AU, r_in=0.11 * AU, r_out=1.85 * AU)
    tab = O.make_ens_table([e])
    p = O.inject(field, tab, 0, np.array([0], dtype=np.uint32))
    gam = 1.0 + 81.0 * KEV / (M_ELECTRON * C_LIGHT ** 2)
    v = p["u"][0] / gam
    assert v / C_LIGHT == pytest.approx(0.5049, abs=2e-4)
    t_coll = 0.5 * AU / v
    assert 400.0 < t_coll < 600.0 and 54.0 / t_coll == pytest.approx(0.1, abs=0.02)
