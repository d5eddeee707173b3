/*
 * gc_oracle.h -- FP64 CPU oracle of the relativistic guiding-centre electron
 * method of Houeibib, Pantellini & Griton (A&A 2025, arXiv 2403.06706).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP library; the only thing the two sides
 * share is the seeded input generator package (fields and injection recipes).
 *
 * Units are SI throughout.  State X = (r, th, ph, u) with u = gamma v_par
 * (Sect. 2.2, X = {R, gamma v_par}), plus the magnetic moment mu_B (Eq. 3:
 * constant between collisions).
 */
#ifndef GC_ORACLE_H
#define GC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_ACTIVE = 0, OR_EXITED = 1, OR_FINISHED = 2, OR_NONFINITE = 3 };
enum { OR_BOOTSTRAP = 1u, OR_PENDING = 2u };
enum { OR_FIELD_GRID = 0, OR_FIELD_PARKER = 1, OR_FIELD_CALLBACK = 2 };

typedef struct {
    int32_t kind;          /* OR_FIELD_GRID or OR_FIELD_PARKER (closed form) */
    int32_t nr, nth, nph;  /* node counts (also used for the theta exit bounds in PARKER mode) */
    double r_min, r_max;   /* m */
    const double *data;    /* GRID: [nr][nth][nph][12] node values, local (r,th,ph) basis */
    double a0;             /* PARKER: B_r r^2 (T m^2) */
    double omega;          /* PARKER: rotation rate (rad/s) */
    double v_wind;         /* PARKER: radial wind speed (m/s) */
    /* CALLBACK: the 12 components at a point from a caller-supplied function
     * (the test suite's FP64 neural field); returns 0 where undefined.  Runs
     * single-threaded: pass nthreads = 1 to the advance calls. */
    int (*eval)(void *user, double r, double th, double ph, double out[12]);
    void *user;
    /* grid fields only: NULL, or [nr][nth][nph][9] node values of (v_E.grad)b,
     * (b.grad)v_E and (v_E.grad)v_E (local basis); with them the full Eqs. 1-2 are
     * integrated, without them the reduced form */
    const double *extra;
} or_field;

typedef struct {
    double ekin;           /* kinetic energy (J) */
    double r0, lat0, lon0; /* injection site (m, rad, rad) */
    double dlon, dr0, dlat;/* half-widths of the uniform spreads */
    double mu_lo, mu_hi;   /* pitch-angle cosine range */
} or_inject_params;

typedef struct {
    double q, m;           /* charge (C), rest mass (kg) */
    double lambda;         /* mean free path along B (m); <= 0: no scattering */
    double r_in, r_out;    /* exit shell (m) */
    uint64_t seed;         /* generator key word 0 */
    uint32_t ensemble;     /* generator key word 1 */
    int32_t drift_free;    /* 1: only v_par b kept in dR/dt (paper Sect. 3.2 diagnostic) */
    int64_t max_steps;     /* > 0: FINISHED after this many steps (counted over all generations) */
    int32_t scatter_law;   /* 0: mu' = 1 - 2a (Eq. 10); 1: mu' = +-sqrt(a) (Eq. 12) */
    int32_t collision_mode;/* 0: exponential free path per collision index; 1: per-step draw (Eq. 9 literally) */
    int64_t rebirth_steps; /* Sect. 3 continuous injection: an exit at a step count below this is a rebirth */
    or_inject_params inj;  /* the injection recipe a reborn particle starts from again */
    double v_wind;         /* > 0: the scattering centres move with a radial wind of this speed (m/s), Sect. 3.3 */
} or_ens;

typedef struct {
    double r, th, ph, u;   /* guiding-centre position, u = gamma v_par */
    double mu_B;           /* magnetic moment (J/T) */
    double fp[4];          /* F^{n-1} */
    double dtp;            /* previous step size (s) */
    double s;              /* path length since the last collision (m) */
    double ell;            /* current free path (m) */
    double t;              /* age: time since the current generation began (s) */
    uint32_t k;            /* collisions so far */
    uint32_t flags;        /* OR_BOOTSTRAP | OR_PENDING */
    uint32_t status;       /* OR_ACTIVE ... */
    uint32_t step;         /* steps taken since the first injection, over all generations */
    uint32_t id;           /* particle id within its ensemble */
    uint32_t ens;          /* index into the ensemble table */
    uint32_t gen;          /* generation: rebirths so far (generator counter word 3) */
    uint32_t birth;        /* step count at which the current generation began */
} or_particle;

typedef struct {
    int32_t depth;         /* entries per particle (0: off) */
    int32_t pad;
    uint32_t *step;        /* [n][depth]: step count at which collision k+1 was applied */
    double *mu_new;        /* [n][depth]: post-collision pitch cosine */
    double *ell;           /* [n][depth]: free path drawn at collision k+1 */
} or_log;

typedef struct {
    int32_t n_rbins;   double r_lo, r_hi;      /* radial bins (active particles) */
    int32_t n_mubins;                          /* pitch-cosine histogram on [-1, 1] */
    double sel_r_lo, sel_r_hi;                 /* radial window for the two histograms below */
    double age_lo, age_hi;                     /* age window for the pitch-cosine histogram */
    int32_t min_collisions;                    /* ... and minimum collision count */
    int32_t n_agebins; double age_max;         /* energy-vs-age histogram: age bins on [0, age_max) */
    int32_t n_ebins;   double e_lo, e_hi;      /* energy bins on [e_lo, e_hi) in units of e_unit */
    double e_unit;                             /* J per energy unit (e.g. 1 eV) */
    double len_unit;                           /* m per length unit for the r sum (e.g. 1 AU) */
    uint32_t min_birth;                        /* binned sums: generation began at step >= min_birth */
} or_moment_spec;

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double or_u01(uint64_t x);

int  or_field_eval(const or_field *f, double r, double th, double ph, double out[12]);
void or_parker_closed_form(double a0, double omega, double v_wind, double r, double th, double out[12]);
void or_rhs(const double X[4], double mu_B, double q, double m, int drift_free,
            const double fld[12], const double *xfld, double F[4], double *vpar, double *gamma);
int  or_field_eval_extra(const or_field *f, double r, double th, double ph, double out[9]);
void or_pc_predict(const double X[4], const double Fn[4], const double Fp[4],
                   double h, double tau, double out[4]);
void or_pc_correct(const double X[4], const double Fn[4], const double Fs[4], const double Fp[4],
                   double h, double tau, double out[4]);

void or_inject(const or_field *f, const or_ens *e, uint32_t ens_index, const uint32_t *ids, int64_t n,
               or_particle *out);
void or_advance(const or_field *f, const or_ens *ens_table, or_particle *p, int64_t n,
                double dt, int64_t n_steps, int nthreads, const or_log *log);
void or_advance_traj(const or_field *f, const or_ens *ens_table, or_particle *p,
                     double dt, int64_t n_steps, double *traj);
int64_t or_moments_size(const or_moment_spec *spec);
void or_moments(const or_field *f, const or_ens *ens_table, const or_particle *p, int64_t n,
                const or_moment_spec *spec, int64_t *out);
int  or_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
