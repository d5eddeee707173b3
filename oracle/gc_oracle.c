/*
 * gc_oracle.c -- plain, slow, FP64 CPU oracle of the relativistic
 * guiding-centre (GC) electron method of Houeibib, Pantellini & Griton
 * (arXiv 2403.06706).  TEST INFRASTRUCTURE ONLY: loaded by the tests, the
 * smoke check and the benchmark's CPU-baseline leg, never by the product path.
 *
 * Each function follows one passage of the paper:
 *   or_field_eval        trilinear interpolation of the gridded field (Sect. 2.2)
 *   or_rhs               GC equations, Eqs. (1)-(3), with the definitions that follow them;
 *                        the terms with derivatives of b and v_E when the field carries them
 *   or_pc_predict/correct third-order predictor-corrector, Eqs. (5)-(6)
 *   bootstrap            backward Euler start at t = 0 and after a collision (Sect. 2.2)
 *   collisions           hard-sphere scattering, Eqs. (9)-(10) (and (12)), in the inertial
 *                        frame (Sect. 3) or in the frame of the wind (Sect. 3.3)
 *   or_inject            injection of Sect. 3
 *   rebirth              continuous injection of Sect. 3: an electron that leaves the
 *                        shell starts again from its initial state
 * Readings of the paper where it is silent or garbled are marked READING.
 */
#include "gc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_C 299792458.0   /* speed of light (m/s) */
#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11), from its definition:  */
/* ten rounds of two 64x64->128 multiplies; key bumped by Weyl constants.    */
/* ------------------------------------------------------------------------ */
static void mulhilo(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    __uint128_t p = (__uint128_t)a * (__uint128_t)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo(M0, c0, &hi0, &lo0);
        mulhilo(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform on [0, 1) from the top 53 bits */
double or_u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* generator block for (particle id, counter word 1, purpose, generation) under
 * key (seed, ensemble) */
static void draw(const or_ens *e, uint32_t id, uint64_t w1, uint64_t purpose, uint32_t gen, double a[4])
{
    uint64_t ctr[4] = { (uint64_t)id, w1, purpose, (uint64_t)gen };
    uint64_t key[2] = { e->seed, (uint64_t)e->ensemble };
    uint64_t o[4];
    or_philox4x64_10(ctr, key, o);
    for (int i = 0; i < 4; ++i) a[i] = or_u01(o[i]);
}

enum { PURPOSE_PATH = 0, PURPOSE_INJECT = 1, PURPOSE_STEPDRAW = 2 };

/* ------------------------------------------------------------------------ */
/* Field: closed-form Parker spiral and trilinear interpolation of a grid.   */
/* ------------------------------------------------------------------------ */
/* Parker spiral B_r = a0/r^2, B_ph = -w B_r with w = omega r sin(th)/v,
 * E = -v r^ x B, and the closed forms of grad|B| and (b.grad)b in the
 * local basis (derived by hand from |B| = B_r sqrt(1+w^2) and b = (1, 0, -w)/sqrt(1+w^2)). */
void or_parker_closed_form(double a0, double omega, double v, double r, double th, double out[12])
{
    double st = sin(th), ct = cos(th);
    double w = omega * r * st / v;
    double w2 = w * w, q = 1.0 + w2;
    double br = a0 / (r * r);
    double bmag = br * sqrt(q);
    double cot = ct / st;
    out[0] = br;  out[1] = 0.0;  out[2] = -w * br;
    out[3] = 0.0; out[4] = v * (-w * br); out[5] = 0.0;           /* E_th = v B_ph */
    out[6] = bmag * (-2.0 / r + w2 / (r * q));
    out[7] = bmag * w2 * cot / (r * q);
    out[8] = 0.0;
    out[9]  = -w2 * (2.0 + w2) / (r * q * q);
    out[10] = -w2 * cot / (r * q);
    out[11] = -w * (2.0 + w2) / (r * q * q);
}

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* returns 1 if every input and output is finite */
/* trilinear interpolation of an [nr][nth][nph][nc] node array */
static void grid_interp(const or_field *f, const double *data, int nc, double r, double th, double ph, double *out)
{
    const int nr = f->nr, nth = f->nth, nph = f->nph;
    const double dr = (f->r_max - f->r_min) / (nr - 1);
    const double dth = OR_PI / nth;
    const double dph = 2.0 * OR_PI / nph;
    /* index-space coordinates: r nodes from r_min, theta nodes cell-centred, phi periodic */
    double x = (r - f->r_min) / dr;
    double y = th / dth - 0.5;
    double z = ph / dph;
    double fi = clampd(floor(x), 0.0, (double)(nr - 2));
    double fj = clampd(floor(y), 0.0, (double)(nth - 2));
    int i = (int)fi, j = (int)fj;
    double wr = clampd(x - fi, 0.0, 1.0);
    double wt = clampd(y - fj, 0.0, 1.0);
    double zf = floor(z);
    double wp = z - zf;
    double km = fmod(zf, (double)nph);
    if (km < 0) km += nph;
    int k0 = (int)km;
    int k1 = (k0 + 1) % nph;
    for (int c = 0; c < nc; ++c) out[c] = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int cc = 0; cc < 2; ++cc) {
                double w = (a ? wr : 1.0 - wr) * (b ? wt : 1.0 - wt) * (cc ? wp : 1.0 - wp);
                size_t node = ((size_t)(i + a) * nth + (size_t)(j + b)) * nph + (size_t)(cc ? k1 : k0);
                const double *v = data + node * nc;
                for (int c = 0; c < nc; ++c) out[c] += w * v[c];
            }
}

int or_field_eval(const or_field *f, double r, double th, double ph, double out[12])
{
    if (!(isfinite(r) && isfinite(th) && isfinite(ph))) return 0;
    if (f->kind == OR_FIELD_PARKER) {
        or_parker_closed_form(f->a0, f->omega, f->v_wind, r, th, out);
    } else if (f->kind == OR_FIELD_CALLBACK) {
        if (!f->eval || !f->eval(f->user, r, th, ph, out)) return 0;
    } else {
        grid_interp(f, f->data, 12, r, th, ph, out);
    }
    for (int c = 0; c < 12; ++c) if (!isfinite(out[c])) return 0;
    return 1;
}

/* The three vectors of the full Eqs. 1-2, (v_E.grad)b, (b.grad)v_E and
 * (v_E.grad)v_E, interpolated like the field; 0 when the field has none. */
int or_field_eval_extra(const or_field *f, double r, double th, double ph, double out[9])
{
    if (f->kind != OR_FIELD_GRID || !f->extra) return 0;
    if (!(isfinite(r) && isfinite(th) && isfinite(ph))) return 0;
    grid_interp(f, f->extra, 9, r, th, ph, out);
    for (int c = 0; c < 9; ++c) if (!isfinite(out[c])) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Guiding-centre right-hand side, Eqs. (1)-(2).                             */
/* ------------------------------------------------------------------------ */
static void cross(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/*
 * F = dX/dt for X = (r, th, ph, u).  Field components are in the orthonormal
 * local basis (r^, th^, ph^), right-handed (r^ x th^ = ph^).
 *   b = B/B, v_E = E x b / B, E_par = E.b,
 *   READING (gamma from the state): gamma = sqrt(1 + u^2/c^2 + 2 mu_B B/(m c^2)),
 *     i.e. p^2 = (m u)^2 + 2 m mu_B B with mu_B = m gamma^2 v_perp^2/(2B) (Sect. 2.2 defs),
 *     v_E neglected in gamma since |u_sw| << c (Sect. 2.2).
 *   dR/dt = v_par b + v_E + (gamma m/(q B)) b x a,
 *     a = mu_B/(gamma^2 m) grad B + (q v_par E_par/(gamma m c^2)) v_E + v_par^2 (b.grad)b
 *     READING: the printed E_par v_E term lacks the factor q/(m c^2) needed for
 *     its dimension (it is the d(gamma)/dt v_E inertia term).
 *     READING: the terms with (v_E.grad)b, (b.grad)v_E and (v_E.grad)v_E need
 *     derivatives of b and v_E that the 12 gridded components do not hold; they are dropped.
 *   du/dt = (q/m) E_par - mu_B/(gamma m) b.grad B + gamma v_E.[v_par (b.grad)b]   (Eq. 2, same reduction)
 *   drift_free: dR/dt = v_par b and du/dt = (q/m) E_par - mu_B/(gamma m) b.grad B
 *   (the "only v_par b retained" runs of Sect. 3.2).
 * Position rates: (V_r, V_th / r, V_ph / (r sin th)).
 */
void or_rhs(const double X[4], double mu_B, double q, double m, int drift_free,
            const double fld[12], const double *xfld, double F[4], double *vpar_out, double *gamma_out)
{
    const double r = X[0], th = X[1], u = X[3];
    const double *Bv = fld, *E = fld + 3, *G = fld + 6, *K = fld + 9;
    double B = sqrt(dot(Bv, Bv));
    double b[3] = { Bv[0] / B, Bv[1] / B, Bv[2] / B };
    double gamma = sqrt(1.0 + (u * u) / (OR_C * OR_C) + 2.0 * mu_B * B / (m * OR_C * OR_C));
    double vpar = u / gamma;
    double Epar = dot(E, b);
    double Exb[3];
    cross(E, b, Exb);
    double vE[3] = { Exb[0] / B, Exb[1] / B, Exb[2] / B };
    double V[3], udot;
    if (drift_free) {
        for (int c = 0; c < 3; ++c) V[c] = vpar * b[c];
        udot = (q / m) * Epar - mu_B / (gamma * m) * dot(b, G);
    } else {
        double a[3], bxa[3];
        for (int c = 0; c < 3; ++c)
            a[c] = mu_B / (gamma * gamma * m) * G[c]
                 + q * vpar * Epar / (gamma * m * OR_C * OR_C) * vE[c]
                 + vpar * vpar * K[c];
        udot = (q / m) * Epar - mu_B / (gamma * m) * dot(b, G) + gamma * vpar * dot(vE, K);
        if (xfld) {
            /* the full Eqs. 1-2: v_par((v_E.grad)b + (b.grad)v_E) + (v_E.grad)v_E in the
             * bracket of dR/dt, gamma v_E.(v_E.grad)b in d(gamma v_par)/dt */
            const double *A = xfld, *Cv = xfld + 3, *D = xfld + 6;
            for (int c = 0; c < 3; ++c) a[c] += vpar * (A[c] + Cv[c]) + D[c];
            udot += gamma * dot(vE, A);
        }
        cross(b, a, bxa);
        double pref = gamma * m / (q * B);
        for (int c = 0; c < 3; ++c) V[c] = vpar * b[c] + vE[c] + pref * bxa[c];
    }
    F[0] = V[0];
    F[1] = V[1] / r;
    F[2] = V[2] / (r * sin(th));
    F[3] = udot;
    if (vpar_out) *vpar_out = vpar;
    if (gamma_out) *gamma_out = gamma;
}

/* ------------------------------------------------------------------------ */
/* Predictor-corrector, Eqs. (5)-(6), with tau = dt^n / dt^{n-1}.            */
/* ------------------------------------------------------------------------ */
void or_pc_predict(const double X[4], const double Fn[4], const double Fp[4],
                   double h, double tau, double out[4])
{
    for (int c = 0; c < 4; ++c)
        out[c] = X[c] + h * ((1.0 + tau / 2.0) * Fn[c] - (tau / 2.0) * Fp[c]);
}

void or_pc_correct(const double X[4], const double Fn[4], const double Fs[4], const double Fp[4],
                   double h, double tau, double out[4])
{
    for (int c = 0; c < 4; ++c)
        out[c] = X[c] + h / (6.0 * (1.0 + tau)) *
                 (3.0 * (Fn[c] + Fs[c]) + 4.0 * tau * (Fn[c] + Fs[c] / 2.0) + tau * tau * (Fn[c] - Fp[c]));
}

/* ------------------------------------------------------------------------ */
/* Injection (Sect. 3) and one particle's time loop.                         */
/* ------------------------------------------------------------------------ */
static double theta_lo(const or_field *f) { return 0.5 * OR_PI / f->nth; }
static double theta_hi(const or_field *f) { return OR_PI - 0.5 * OR_PI / f->nth; }

static int outside(const or_field *f, const or_ens *e, double r, double th)
{
    return r < e->r_in || r > e->r_out || th < theta_lo(f) || th > theta_hi(f);
}

static double free_path(const or_ens *e, double a)
{
    /* exponential free path of mean lambda (READING of Eq. 9: P(no collision over a path s) = exp(-s/lambda)) */
    return e->lambda > 0.0 ? -e->lambda * log(1.0 - a) : INFINITY;
}

/* Initial state of particle id, generation gen (Sect. 3): released at the
 * injection site with the recipe's energy and pitch.  Site and pitch come from
 * the block (id, 0, inject, 0), the same for every generation (READING: a reborn
 * electron restarts on the same line with the same initial velocity, so with
 * its own initial state); the first free path from the block (id, 0, path, gen). */
static void init_particle(const or_field *f, const or_ens *e, uint32_t id, uint32_t gen, or_particle *p)
{
    const or_inject_params *ip = &e->inj;
    double a[4];
    draw(e, id, 0, PURPOSE_INJECT, 0, a);
    p->ph = ip->lon0 + ip->dlon * (2.0 * a[0] - 1.0);
    double mup = ip->mu_lo + (ip->mu_hi - ip->mu_lo) * a[1];
    p->r = ip->r0 + ip->dr0 * (2.0 * a[2] - 1.0);
    double lat = ip->lat0 + ip->dlat * (2.0 * a[3] - 1.0);
    p->th = 0.5 * OR_PI - lat;                 /* READING: magnetic latitude = heliographic latitude (aligned dipole) */
    double gamma = 1.0 + ip->ekin / (e->m * OR_C * OR_C);
    double pmom = e->m * OR_C * sqrt(gamma * gamma - 1.0);
    p->u = pmom * mup / e->m;
    p->flags = OR_BOOTSTRAP;
    p->status = OR_ACTIVE;
    double b[4];
    draw(e, id, 0, PURPOSE_PATH, gen, b);
    p->ell = free_path(e, b[0]);
    if (outside(f, e, p->r, p->th)) { p->status = OR_EXITED; return; }
    double fld[12];
    if (!or_field_eval(f, p->r, p->th, p->ph, fld)) { p->status = OR_NONFINITE; return; }
    double B = sqrt(fld[0] * fld[0] + fld[1] * fld[1] + fld[2] * fld[2]);
    p->mu_B = pmom * pmom * (1.0 - mup * mup) / (2.0 * e->m * B);
}

void or_inject(const or_field *f, const or_ens *e, uint32_t ens_index, const uint32_t *ids, int64_t n,
               or_particle *out)
{
    for (int64_t i = 0; i < n; ++i) {
        or_particle *p = &out[i];
        memset(p, 0, sizeof(*p));
        p->id = ids[i];
        p->ens = ens_index;
        init_particle(f, e, p->id, 0, p);
    }
}

/* Rebirth (Sect. 3): the electron that just left the shell is released again
 * at once, as generation gen + 1, with age 0 and no collisions; the global step
 * count goes on.  Its collision-log row starts again empty. */
static void rebirth(const or_field *f, const or_ens *e, or_particle *p, const or_log *log, int64_t pi)
{
    const uint32_t id = p->id, ens = p->ens, step = p->step, gen = p->gen + 1;
    memset(p, 0, sizeof(*p));
    p->id = id;
    p->ens = ens;
    p->step = step;
    p->gen = gen;
    p->birth = step;
    init_particle(f, e, id, gen, p);
    if (log && log->depth > 0) {
        for (int32_t j = 0; j < log->depth; ++j) {
            size_t idx = (size_t)pi * log->depth + j;
            log->step[idx] = 0xFFFFFFFFu;
            log->mu_new[idx] = NAN;
            log->ell[idx] = NAN;
        }
    }
}

/* Component of the wind velocity along b.  READING (Sect. 3.3): the wind is
 * radial with speed v_wind, as in the stand-in fields; its component across B
 * is the E x B drift the guiding centre already moves with, so the frame of
 * the scattering centres differs from the drift frame by V_par = v_wind b_r. */
static double wind_par(const or_ens *e, const double fld[12])
{
    double B = sqrt(fld[0] * fld[0] + fld[1] * fld[1] + fld[2] * fld[2]);
    return e->v_wind * fld[0] / B;
}

/* Path covered along b in one step, against the scattering centres (READING of
 * Eq. 9: the trapezoid of the speed along b at X^n and X*).  Inertial frame:
 * |v_par|.  Wind frame: the centres move with V_par along b, and a boost along
 * b turns dx - V_par dt into Gamma (v_par - V_par) dt. */
static double path_step(const or_ens *e, double vpn, const double gn[12], double vps, const double gs[12], double dt)
{
    if (e->v_wind > 0.0) {
        double Vn = wind_par(e, gn), Vs = wind_par(e, gs);
        double Gn = 1.0 / sqrt(1.0 - Vn * Vn / (OR_C * OR_C));
        double Gs = 1.0 / sqrt(1.0 - Vs * Vs / (OR_C * OR_C));
        return 0.5 * (Gn * fabs(vpn - Vn) + Gs * fabs(vps - Vs)) * dt;
    }
    return 0.5 * (fabs(vpn) + fabs(vps)) * dt;
}

/* hard-sphere collision number k (Eqs. 9-10): new pitch cosine drawn in the
 * frame of the scattering centres, |p| kept there, new free path; the position
 * is unchanged.  Inertial centres (Sect. 3): |p| kept.  Wind-frame centres
 * (Sect. 3.3): the momentum (p_par, p_perp) and energy are boosted along b by
 * V_par (a Lorentz boost: p_perp unchanged), the collision keeps |p~| and sets
 * p~_par = mu' |p~|, and the boost back gives the new p_par and p_perp. */
static void collide(const or_ens *e, or_particle *p, const double fld[12], const or_log *log, int64_t pi)
{
    double B = sqrt(fld[0] * fld[0] + fld[1] * fld[1] + fld[2] * fld[2]);
    p->k += 1;
    double a[4];
    draw(e, p->id, p->k, PURPOSE_PATH, p->gen, a);
    double m = e->m;
    double mun;
    if (e->scatter_law == 1) mun = (a[2] < 0.5 ? -1.0 : 1.0) * sqrt(a[1]);   /* Eq. 12 */
    else mun = 1.0 - 2.0 * a[1];                                              /* Eq. 10 */
    double ppar = m * p->u;
    double pperp2 = 2.0 * m * p->mu_B * B;
    if (e->v_wind > 0.0) {
        double V = wind_par(e, fld);
        double G = 1.0 / sqrt(1.0 - V * V / (OR_C * OR_C));
        double En = sqrt(m * m * OR_C * OR_C * OR_C * OR_C + (ppar * ppar + pperp2) * OR_C * OR_C);
        double pw = G * (ppar - V * En / (OR_C * OR_C));          /* p~_par */
        double Ew = G * (En - V * ppar);                          /* E~ */
        double P2 = pw * pw + pperp2;                             /* |p~|^2, kept */
        double pw_new = mun * sqrt(P2);
        p->u = G * (pw_new + V * Ew / (OR_C * OR_C)) / m;
        p->mu_B = P2 * (1.0 - mun * mun) / (2.0 * m * B);
    } else {
        double p2 = ppar * ppar + pperp2;
        p->u = mun * sqrt(p2) / m;
        p->mu_B = p2 * (1.0 - mun * mun) / (2.0 * m * B);
    }
    p->ell = free_path(e, a[0]);
    p->s = 0.0;
    p->flags = (p->flags | OR_BOOTSTRAP) & ~OR_PENDING;
    if (log && log->depth > 0 && p->k <= (uint32_t)log->depth) {
        size_t idx = (size_t)pi * log->depth + (p->k - 1);
        log->step[idx] = p->step;
        log->mu_new[idx] = mun;
        log->ell[idx] = p->ell;
    }
}

static int finite4(const double X[4])
{
    return isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2]) && isfinite(X[3]);
}

static void advance_one(const or_field *f, const or_ens *e, or_particle *p, double dt, int64_t n_steps,
                        const or_log *log, int64_t pi, double *traj)
{
    const int full = f->kind == OR_FIELD_GRID && f->extra != NULL;   /* full Eqs. 1-2 */
    for (int64_t it = 0; it < n_steps; ++it) {
        if (p->status != OR_ACTIVE) return;
        double X[4] = { p->r, p->th, p->ph, p->u };
        double g[12];
        if (!or_field_eval(f, X[0], X[1], X[2], g)) { p->status = OR_NONFINITE; return; }
        if (p->flags & OR_PENDING) {
            collide(e, p, g, log, pi);
            X[3] = p->u;
        }
        double Fn[4], vpn, gam, xg[9];
        const double *xn = full ? (or_field_eval_extra(f, X[0], X[1], X[2], xg) ? xg : NULL) : NULL;
        if (full && !xn) { p->status = OR_NONFINITE; return; }
        or_rhs(X, p->mu_B, e->q, e->m, e->drift_free, g, xn, Fn, &vpn, &gam);
        double Fp[4], tau;
        if (p->flags & OR_BOOTSTRAP) {
            /* X^{n-1} = X^n - dt F^n, F^{n-1} = F(X^{n-1}) (Sect. 2.2) */
            double Xm[4], gm[12];
            for (int c = 0; c < 4; ++c) Xm[c] = X[c] - dt * Fn[c];
            if (!or_field_eval(f, Xm[0], Xm[1], Xm[2], gm)) { p->status = OR_NONFINITE; return; }
            double xm[9];
            if (full && !or_field_eval_extra(f, Xm[0], Xm[1], Xm[2], xm)) { p->status = OR_NONFINITE; return; }
            or_rhs(Xm, p->mu_B, e->q, e->m, e->drift_free, gm, full ? xm : NULL, Fp, NULL, NULL);
            tau = 1.0;
            p->flags &= ~OR_BOOTSTRAP;
        } else {
            for (int c = 0; c < 4; ++c) Fp[c] = p->fp[c];
            tau = dt / p->dtp;
        }
        double Xs[4], gs[12], Fs[4], vps;
        or_pc_predict(X, Fn, Fp, dt, tau, Xs);
        if (!or_field_eval(f, Xs[0], Xs[1], Xs[2], gs)) { p->status = OR_NONFINITE; return; }
        double xs[9];
        if (full && !or_field_eval_extra(f, Xs[0], Xs[1], Xs[2], xs)) { p->status = OR_NONFINITE; return; }
        or_rhs(Xs, p->mu_B, e->q, e->m, e->drift_free, gs, full ? xs : NULL, Fs, &vps, NULL);
        double Xn[4];
        or_pc_correct(X, Fn, Fs, Fp, dt, tau, Xn);
        double ds = path_step(e, vpn, g, vps, gs, dt);
        if (e->lambda > 0.0) {
            if (e->collision_mode == 1) {
                double a[4];
                draw(e, p->id, p->step, PURPOSE_STEPDRAW, p->gen, a);
                if (a[0] < 1.0 - exp(-ds / e->lambda)) p->flags |= OR_PENDING;
            } else {
                p->s += ds;
                if (p->s >= p->ell) p->flags |= OR_PENDING;
            }
        }
        p->r = Xn[0]; p->th = Xn[1]; p->ph = Xn[2]; p->u = Xn[3];
        for (int c = 0; c < 4; ++c) p->fp[c] = Fn[c];
        p->dtp = dt;
        p->t += dt;
        p->step += 1;
        if (traj) for (int c = 0; c < 4; ++c) traj[(it + 1) * 4 + c] = Xn[c];
        if (!finite4(Xn)) { p->status = OR_NONFINITE; return; }
        if (outside(f, e, p->r, p->th)) {
            if ((int64_t)p->step >= e->rebirth_steps) { p->status = OR_EXITED; return; }
            rebirth(f, e, p, log, pi);
            if (p->status != OR_ACTIVE) return;
        }
        if (e->max_steps > 0 && p->step >= (uint64_t)e->max_steps) { p->status = OR_FINISHED; return; }
    }
}

void or_advance(const or_field *f, const or_ens *ens_table, or_particle *p, int64_t n,
                double dt, int64_t n_steps, int nthreads, const or_log *log)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
#endif
    for (int64_t i = 0; i < n; ++i)
        advance_one(f, &ens_table[p[i].ens], &p[i], dt, n_steps, log, i, NULL);
}

void or_advance_traj(const or_field *f, const or_ens *ens_table, or_particle *p,
                     double dt, int64_t n_steps, double *traj)
{
    traj[0] = p->r; traj[1] = p->th; traj[2] = p->ph; traj[3] = p->u;
    for (int64_t it = 1; it <= n_steps; ++it)
        for (int c = 0; c < 4; ++c) traj[it * 4 + c] = NAN;
    advance_one(f, &ens_table[p->ens], p, dt, n_steps, NULL, 0, traj);
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Moments (snapshot statistics of Sect. 3: <sin^2 alpha>(r), energy vs age, */
/* pitch-cosine distributions) as integer and fixed-point sums.              */
/* ------------------------------------------------------------------------ */
int64_t or_moments_size(const or_moment_spec *s)
{
    return 8 + 3 * (int64_t)s->n_rbins + s->n_mubins + (int64_t)s->n_agebins * s->n_ebins;
}

static int64_t fix(double x, double scale) { return (int64_t)floor(x * scale); }

void or_moments(const or_field *f, const or_ens *ens_table, const or_particle *p, int64_t n,
                const or_moment_spec *s, int64_t *out)
{
    const int64_t nout = or_moments_size(s);
    memset(out, 0, (size_t)nout * sizeof(int64_t));
    int64_t *rb = out + 8;
    int64_t *mh = rb + 3 * (int64_t)s->n_rbins;
    int64_t *eh = mh + s->n_mubins;
    for (int64_t i = 0; i < n; ++i) {
        const or_particle *q = &p[i];
        const or_ens *e = &ens_table[q->ens];
        if (q->status <= OR_NONFINITE) out[q->status] += 1;
        out[4] += q->k;
        out[5] += q->step;
        if (q->status != OR_ACTIVE) continue;
        out[6] += fix(q->r / s->len_unit, 4294967296.0);
        if (q->k >= 1) out[7] += 1;
        if (q->birth < s->min_birth) continue;          /* Sect. 3: only particles injected after a given time */
        double g[12];
        if (!or_field_eval(f, q->r, q->th, q->ph, g)) continue;
        double B = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        double m = e->m;
        double p2 = (m * q->u) * (m * q->u) + 2.0 * m * q->mu_B * B;   /* |p|^2 */
        double pm = sqrt(p2);
        double mu = pm > 0.0 ? (m * q->u) / pm : 1.0;                   /* pitch-angle cosine */
        double sin2 = 1.0 - mu * mu;
        double gamma = sqrt(1.0 + p2 / (m * m * OR_C * OR_C));
        double ekin = (gamma - 1.0) * m * OR_C * OR_C / s->e_unit;
        if (s->n_rbins > 0) {
            double x = (q->r - s->r_lo) / (s->r_hi - s->r_lo) * s->n_rbins;
            if (x >= 0.0 && x < s->n_rbins) {
                int64_t bi = (int64_t)floor(x);
                rb[3 * bi + 0] += 1;
                rb[3 * bi + 1] += fix(sin2, 4294967296.0);
                rb[3 * bi + 2] += fix(ekin, 65536.0);
            }
        }
        if (q->r < s->sel_r_lo || q->r >= s->sel_r_hi) continue;
        if (s->n_mubins > 0 && q->t >= s->age_lo && q->t < s->age_hi && q->k >= (uint32_t)s->min_collisions) {
            double x = (mu + 1.0) * 0.5 * s->n_mubins;
            int64_t bi = (int64_t)floor(x);
            if (bi < 0) bi = 0;
            if (bi >= s->n_mubins) bi = s->n_mubins - 1;
            mh[bi] += 1;
        }
        if (s->n_agebins > 0 && s->n_ebins > 0) {
            double xa = q->t / s->age_max * s->n_agebins;
            double xe = (ekin - s->e_lo) / (s->e_hi - s->e_lo) * s->n_ebins;
            if (xa >= 0.0 && xa < s->n_agebins && xe >= 0.0 && xe < s->n_ebins)
                eh[(int64_t)floor(xa) * s->n_ebins + (int64_t)floor(xe)] += 1;
        }
    }
}
