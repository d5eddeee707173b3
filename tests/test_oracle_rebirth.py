"""Pins of the oracle's continuous injection (Sect. 3): an electron that leaves
the shell is reborn at once from its initial state; generations draw fresh
free paths; snapshots of a reborn population hold every electron.

The pins rest on facts other than the oracle's own code: without scattering, in
a radial field of constant strength, an electron released along B moves
outward at constant speed, so each generation must retrace the first one
exactly and rebirths must come every n_exit steps; with rebirth on, the number
of live electrons is a constant of the run, which fixes the sample count of
accumulated snapshots (the paper's 9.4e6 figure); free paths of every
generation must be exponential with mean lambda (Eq. 9)."""
import math

import numpy as np
from scipy import stats

import oracle as O
from synthetic import AU, SphericalGrid, fields
from synthetic.workloads import Ensemble

G = SphericalGrid(16, 8, 8, 0.1 * AU, 2.0 * AU)
STRAIGHT = fields.straight(G)
FIELD = O.Field(G, STRAIGHT)


def _ens(**kw):
    base = dict(n=64, ensemble=1, seed=5, r0=0.5 * AU, lat0=0.0, dlon=0.3, dr0=0.05 * AU, mu_lo=1.0, mu_hi=1.0,
                lambda_par=0.0, r_in=0.11 * AU, r_out=0.8 * AU)
    base.update(kw)
    return Ensemble(**base)


def _inject(e, n=None):
    tab = O.make_ens_table([e])
    p = O.inject(FIELD, tab, 0, np.arange(e.n if n is None else n, dtype=np.uint32))
    return p, tab


def _exit_steps(e, dt):
    """Steps each electron of the first generation takes to leave the shell."""
    p, tab = _inject(e)
    O.advance(FIELD, tab, p, dt, 100000)
    assert np.all(p["status"] == O.EXITED)
    return p["step"].astype(np.int64)


def test_each_generation_retraces_the_first():
    """No scattering, radial field of constant strength, pitch cosine 1: the
    motion is the same in every generation, so after S steps electron i is in
    generation S // n_i, born at step (S // n_i) n_i, in the state the first
    generation had S mod n_i steps after injection (bit for bit: a rebirth
    resets age, history and bootstrap, and the integrator sees the same
    numbers)."""
    dt = 20.0
    e = _ens()
    n_exit = _exit_steps(e, dt)
    assert n_exit.min() > 10 and len(np.unique(n_exit)) > 3     # the radial spread gives different periods
    S = int(3 * n_exit.max() + 7)
    er = _ens(rebirth_steps=10 ** 6)
    p, tab = _inject(er)
    O.advance(FIELD, tab, p, dt, S)
    assert np.all(p["status"] == O.ACTIVE) and np.all(p["step"] == S)
    gen = S // n_exit
    assert np.array_equal(p["gen"].astype(np.int64), gen)
    assert np.array_equal(p["birth"].astype(np.int64), gen * n_exit)
    for i in range(e.n):
        q, qtab = _inject(e)
        q = q[i:i + 1].copy()
        m = int(S - gen[i] * n_exit[i])
        O.advance(FIELD, qtab, q, dt, m)
        for k in ("r", "th", "ph", "u", "mu_B", "fp", "dtp", "s", "t", "k", "flags", "status"):
            assert np.array_equal(p[k][i], q[k][0]), (i, k, p[k][i], q[k][0])


def test_rebirth_window_edge():
    """An exit at step count n is a rebirth iff n < rebirth_steps."""
    dt = 20.0
    e = _ens(n=8, dr0=0.0)
    n_exit = _exit_steps(e, dt)
    n0 = int(n_exit[0])
    assert np.all(n_exit == n0)
    for rb, reborn in ((n0, False), (n0 + 1, True)):
        p, tab = _inject(_ens(n=8, dr0=0.0, rebirth_steps=rb))
        O.advance(FIELD, tab, p, dt, n0 + 5)
        if reborn:
            assert np.all(p["status"] == O.ACTIVE) and np.all(p["gen"] == 1) and np.all(p["birth"] == n0)
            assert np.all(p["step"] == n0 + 5)
        else:
            assert np.all(p["status"] == O.EXITED) and np.all(p["gen"] == 0) and np.all(p["step"] == n0)


def test_population_conserved_and_snapshot_sample_count():
    """With rebirth on for the whole run every snapshot holds all N electrons,
    so S accumulated snapshots give N S samples.  The paper's run (10^3
    electrons, snapshots every 100 steps of 0.54 s from 8.3 h to 150 h) gives
    some 9.4e6; a scaled run of the oracle must give exactly N S."""
    paper = 1000 * math.floor((150.0 - 8.3) * 3600.0 / (100 * 0.54))
    assert round(paper / 1e5) == 94
    e = _ens(n=200, mu_lo=-1.0, mu_hi=1.0, lambda_par=0.05 * AU, rebirth_steps=10 ** 6)
    p, tab = _inject(e)
    spec = O.MomentSpec(n_rbins=8, r_lo=0.1 * AU, r_hi=0.9 * AU)
    acc = np.zeros(O.moments_size(spec), dtype=np.int64)
    S = 40
    for _ in range(S):
        O.advance(FIELD, tab, p, 20.0, 25)
        acc += O.moments(FIELD, tab, p, spec)
    assert acc[0] == e.n * S and acc[1] == 0 and acc[3] == 0
    assert acc[8:8 + 3 * 8:3].sum() == e.n * S          # every sample falls in a radial bin of the shell
    assert p["gen"].sum() > e.n                         # many rebirths took place
    # once the window closes the population drains
    e2 = _ens(n=200, mu_lo=-1.0, mu_hi=1.0, lambda_par=0.05 * AU, rebirth_steps=500)
    p2, tab2 = _inject(e2)
    O.advance(FIELD, tab2, p2, 20.0, 3000)
    assert np.sum(p2["status"] == O.EXITED) > 0
    assert np.all(p2["step"][p2["status"] == O.EXITED] >= 500)


def test_every_generation_draws_exponential_free_paths():
    """Free paths of reborn generations: exponential with mean lambda, and drawn
    from the generation's own stream (counter word 3 = generation)."""
    lam = 0.05 * AU
    e = _ens(n=3000, mu_lo=-1.0, mu_hi=1.0, lambda_par=lam, r_out=0.56 * AU, dr0=0.0, rebirth_steps=10 ** 6)
    p, tab = _inject(e)
    drawn, checked = [], 0
    for _ in range(300):
        O.advance(FIELD, tab, p, 20.0, 1)
        fresh = np.nonzero((p["gen"] >= 1) & (p["t"] == 0.0))[0]    # reborn at the end of this step
        drawn.append(p["ell"][fresh] / lam)
        for i in fresh[:2]:
            a0 = O.u01(O.philox([int(p["id"][i]), 0, 0, int(p["gen"][i])], [e.seed, e.ensemble])[0])
            assert p["ell"][i] == -lam * math.log(1.0 - a0)
            checked += 1
    ell = np.concatenate(drawn)
    assert len(ell) > 1000 and checked > 50
    assert stats.kstest(ell, "expon").pvalue > 0.01
    assert abs(ell.mean() - 1.0) < 3.0 / math.sqrt(len(ell))


def test_moments_birth_selection():
    """Binned sections count only electrons of generations born at or after
    min_birth; the status counts and sums count every electron."""
    e = _ens(n=300, mu_lo=-1.0, mu_hi=1.0, lambda_par=0.05 * AU, rebirth_steps=10 ** 6)
    p, tab = _inject(e)
    O.advance(FIELD, tab, p, 20.0, 400)
    base = dict(n_rbins=8, r_lo=0.1 * AU, r_hi=0.9 * AU, n_mubins=10, sel_r_lo=0.1 * AU, sel_r_hi=0.9 * AU,
                age_lo=0.0, age_hi=1e12, n_agebins=4, age_max=1e5, n_ebins=4, e_lo=0.0, e_hi=1e6)
    all_ = O.moments(FIELD, tab, p, O.MomentSpec(**base))
    cut = 200
    sel = O.moments(FIELD, tab, p, O.MomentSpec(min_birth=cut, **base))
    assert np.array_equal(all_[:8], sel[:8])
    keep = p["birth"] >= cut
    assert 0 < keep.sum() < e.n
    assert sel[8:8 + 3 * 8:3].sum() == keep.sum()
    sub = O.moments(FIELD, tab, p[keep].copy(), O.MomentSpec(**base))
    assert np.array_equal(sel[8:], sub[8:])
