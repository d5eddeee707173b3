/*
 * gcpush.h -- C ABI of the MI355X (gfx950) guiding-centre electron pusher.
 *
 * The library advances relativistic guiding-centre (GC) electrons through a
 * steady gridded spherical field, following Houeibib, Pantellini & Griton,
 * "Dynamics of energetic electrons scattered in the solar wind" (A&A 2025,
 * arXiv 2403.06706):
 *   - GC equations of motion, Eqs. (1)-(3) of Sect. 2.2, with X = (R, gamma v_par);
 *   - field at the particle by trilinear interpolation of the grid (Sect. 2.2);
 *   - third-order predictor-corrector, Eqs. (5)-(6), started by a backward
 *     Euler step at injection and after each collision (Sect. 2.2);
 *   - hard-sphere scattering along the field line, Eqs. (9)-(10) (and (12))
 *     of Sect. 2.3, in the inertial frame (Sect. 3).
 *
 * Conventions (all entry points):
 *   - Every call returns a gc_status and never throws.  Argument errors are
 *     detected on the host before any device work and described by
 *     gc_last_error().  A failed HIP call or launch returns GC_EDEVICE; after
 *     one from gc_advance or gc_advance_graph the particle state may be part
 *     way through a chunk: reload it (gc_set_state) or destroy the context.
 *   - Device work is queued on the context's HIP stream and returns without
 *     waiting, unless stated otherwise.
 *   - Units are SI.  Field vectors are in the local orthonormal spherical
 *     basis (r^, th^, ph^), right-handed.
 *   - The library owns the particle state, the packed field and its scratch
 *     buffers: device memory from the caller's allocator (gc_options.dev_alloc
 *     / dev_free, e.g. a framework's caching allocator), else from hipMalloc.
 *     Buffers passed in are owned by the caller.
 *   - Per-particle faults (leaving the shell, non-finite values) are particle
 *     status values, not errors.
 *   - One context must not be used from two host threads at once.
 */
#ifndef GCPUSH_H
#define GCPUSH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gc_ctx gc_ctx;

typedef enum {
    GC_OK = 0,
    GC_EINVAL = -1,   /* invalid argument (nothing was queued) */
    GC_ENOMEM = -2,   /* device allocation failed */
    GC_EDEVICE = -3,  /* HIP runtime or kernel launch error */
    GC_ESTATE = -4    /* call out of order (e.g. gc_advance before gc_load_field) */
} gc_status;

typedef enum { GC_F64 = 0, GC_F32 = 1, GC_F16 = 2 } gc_dtype;

/* Arithmetic of the push (the paper fixes none):
 *   GC_PREC_F64        everything in FP64;
 *   GC_PREC_F32_ACC64  field interpolation and right-hand side in FP32, position,
 *                      u and time accumulated in FP64;
 *   GC_PREC_F32_KAHAN  everything in FP32, position, u and time accumulated with
 *                      Kahan compensation (compensation terms kept in the state). */
typedef enum { GC_PREC_F64 = 0, GC_PREC_F32_ACC64 = 1, GC_PREC_F32_KAHAN = 2 } gc_precision;

/* particle status */
enum { GC_ACTIVE = 0, GC_EXITED = 1, GC_FINISHED = 2, GC_NONFINITE = 3 };
/* particle flags; bits GC_FLAG_GEN_SHIFT.. hold the generation (rebirths so far) */
enum { GC_FLAG_BOOTSTRAP = 1u, GC_FLAG_PENDING = 2u, GC_FLAG_GEN_SHIFT = 8 };

/* Particle reordering before each chunk of steps. */
enum {
    GC_ORDER_NONE = 0,     /* never reorder; every slot is visited by every launch */
    GC_ORDER_COMPACT = 1,  /* stable partition: active particles first (wavefront ballots) */
    GC_ORDER_BIN = 2       /* radix sort by field cell, inactive particles last */
};

typedef struct {
    void *hip_stream;       /* hipStream_t for all device work; NULL: the null stream */
    int32_t device;         /* HIP device ordinal */
    int32_t precision;      /* gc_precision */
    int32_t order;          /* GC_ORDER_* */
    int32_t chunk_steps;    /* steps per push launch (and per reorder); > 0 */
    int32_t bin_coarsen;    /* cells per bin along each axis = 2^bin_coarsen (GC_ORDER_BIN) */
    int32_t block_size;     /* push workgroup size: 64 (default), 128 or 256; the four-lanes-per-particle
                               form always runs 256-thread workgroups */
    int32_t persistent;     /* 1: persistent push with a tile work queue */
    int32_t tile;           /* particles per work-queue tile (persistent mode, multiple of block_size) */
    int32_t log_depth;      /* per particle, record the step of the first log_depth collisions (0: off) */
    int32_t timing;         /* 1: HIP events on each push launch and each reorder (gc_get_counters);
                               2: on the push launches only (reorder_ms stays 0; each timed
                               dispatch idles the queue a few microseconds) */
    int32_t field_source;   /* GC_SOURCE_GRID (trilinear grid) or GC_SOURCE_MLP (neural field, gc_mlp_set) */
    int32_t tail_threshold; /* grid form, eager gc_advance: chunks whose live count (as read back from an
                               earlier reorder) is below this reorder only every 8 chunks and use a
                               latency form of the push (every field load of a gather in flight;
                               below a quarter of it, four lanes per particle); 0 disables.
                               Persistent form (also in gc_advance_graph): the device picks the same
                               forms from the live count of the chunk's reorder.
                               Results are bitwise identical in every form.  While it is > 0,
                               gc_advance keeps the host at most 3 chunks ahead of the device
                               (it waits for the chunk it issued 3 chunks earlier), so that the
                               live count it reads back is recent. */
    /* Device memory of the context: dev_alloc(bytes, user) returns device memory
     * of that size or NULL, dev_free(ptr, user) releases it; both NULL: hipMalloc
     * and hipFree.  Given together or not at all (GC_EINVAL); fixed at gc_create
     * (gc_set_options keeps them).  The library synchronizes its stream before
     * it releases memory its queued work may still use. */
    void *(*dev_alloc)(size_t bytes, void *user);
    void (*dev_free)(void *ptr, void *user);
    void *alloc_user;
} gc_options;

enum { GC_SOURCE_GRID = 0, GC_SOURCE_MLP = 1 };

/* Fill *opt with the defaults: FP64, cell binning (bin_coarsen 0) every 64
 * steps, 64-thread workgroups, grid form (not persistent; tile 1024), no
 * collision log, no timing, trilinear grid field, tail_threshold 131072,
 * device memory from hipMalloc, the null stream, device 0. */
void gc_default_options(gc_options *opt);

/* Create a context on opt->device.  out receives the handle. */
gc_status gc_create(gc_ctx **out, const gc_options *opt);
void gc_destroy(gc_ctx *ctx);
/* Text of the last error on this context ("" if none).  Valid until the next call. */
const char *gc_last_error(const gc_ctx *ctx);
/* Change options between calls (precision, order, chunk, block, persistence, tile, timing).
 * log_depth and device cannot change after creation. */
gc_status gc_set_options(gc_ctx *ctx, const gc_options *opt);
gc_status gc_get_options(const gc_ctx *ctx, gc_options *opt);

/* ---------------------------------------------------------------- field */
/* Grid geometry (a uniform stand-in for the paper's MHD grid, Sect. 2.1):
 *   r_i  = r_min + i (r_max - r_min)/(nr - 1)   i = 0..nr-1
 *   th_j = (j + 1/2) pi / nth                   j = 0..nth-1
 *   ph_k = 2 pi k / nph  (periodic)             k = 0..nph-1
 * data: HOST pointer to [nr][nth][nph][12] values of type src_dtype, components
 *   B_r B_th B_ph | E_r E_th E_ph | (grad|B|)_r,th,ph | ((b.grad)b)_r,th,ph.
 * The library copies and repacks the data in store_dtype (GC_F16 stores each
 * component divided by a per-component power-of-two scale); the caller's buffer
 * may be freed when the call returns.  The call waits for the upload.  For
 * GC_F32 and GC_F64 stores it keeps a second copy as node records for its
 * four-lanes-per-particle form (device memory about twice the packed field).
 * Non-finite values are allowed: an electron whose field evaluation meets one
 * ends GC_NONFINITE.  (The call scans the data once on the host; a grid whose
 * values are all finite and at most 1e30 in magnitude lets the push skip that
 * test, with the same results.)
 * extra: NULL (the reduced Eqs. 1-2, dropping the terms with derivatives of b
 *   and v_E), or a HOST pointer to [nr][nth][nph][9] values of src_dtype:
 *   (v_E.grad)b | (b.grad)v_E | (v_E.grad)v_E, local basis, v_E = E x B / B^2;
 *   with it every push integrates the full Eqs. 1-2: v_par((v_E.grad)b +
 *   (b.grad)v_E) + (v_E.grad)v_E is added to the bracket of dR/dt and
 *   gamma v_E.(v_E.grad)b to d(gamma v_par)/dt (not in the drift-free form).
 *   Stored like the field (same layout, 3 zero components); the push then
 *   makes a second gather at each evaluation and uses no quad form.  Not
 *   supported with the network field source (GC_EINVAL from gc_advance).
 * Errors: GC_EINVAL if nr < 2, nth < 2, nph < 2, r_min <= 0, r_max <= r_min,
 * data == NULL, a dtype is unknown, or the packed field exceeds 4 GiB (about
 * nr nth (nph + 1) x 48 bytes for GC_F32, 96 for GC_F64, 24 for GC_F16; the
 * gathers use 32-bit byte offsets).  Loading a new field keeps the particles. */
typedef struct {
    int32_t nr, nth, nph;
    int32_t src_dtype;      /* GC_F64 or GC_F32 */
    double r_min, r_max;    /* m */
    const void *data;       /* host */
    int32_t store_dtype;    /* GC_F64, GC_F32 or GC_F16 */
    int32_t pad;
    const void *extra;      /* host or NULL: the full-equation terms, see above */
} gc_field_desc;

gc_status gc_load_field(gc_ctx *ctx, const gc_field_desc *desc);

/* ------------------------------------------------------------ injection */
/* Append desc->n particles of one ensemble (Sect. 3: mono-energetic electrons
 * released at one site).  Particle j of the call gets id first_id + j within
 * the ensemble and the next global index.  Its draws come from Philox4x64-10
 * with key (seed, ensemble) and counter (id, 0, 1, 0):
 *   ph  = lon0 + dlon (2 a0 - 1),  pitch cosine mu = mu_lo + (mu_hi - mu_lo) a1,
 *   r   = r0 + dr0 (2 a2 - 1),     th = pi/2 - (lat0 + dlat (2 a3 - 1)),
 * and its first free path from counter (id, 0, 0, 0): ell_0 = -lambda ln(1 - a0).
 * u = gamma v mu from ekin; mu_B/m = (p/m)^2 (1 - mu^2) / (2 |B(R0)|).
 * A particle placed outside [r_in, r_out] x [th_0, th_{nth-1}] is EXITED.
 * Continuous injection (Sect. 3): a particle that leaves the shell at the end of
 * a step whose step count (counted from its first injection, over all
 * generations) is below rebirth_steps is reborn at once, in the same step:
 * generation g + 1 starts from the same initial state (counter (id, 0, 1, 0)
 * again), with age t = 0, no collisions, a bootstrap start, the state field
 * birth set to that step count, and draws from counter word 3 = g + 1 (first
 * free path (id, 0, 0, g + 1), collision k (id, k, 0, g + 1)).  Its collision
 * log row is cleared.  rebirth_steps <= 0 turns rebirth off; at most 2^24; not
 * supported with the network field source (GC_EINVAL from gc_advance).
 * Scattering in the wind frame (Sect. 3.3, adiabatic cooling): with v_wind > 0
 * the scattering centres move with a radial wind of that speed.  Its component
 * across B is the E x B drift of the guiding centre; along b it is
 * V = v_wind b_r.  A collision boosts (p_par, energy) along b by V (Lorentz;
 * p_perp unchanged), keeps |p~| there, sets p~_par = mu' |p~| and boosts back;
 * the path of Eq. 9 is measured against the centres, Gamma |v_par - V| dt.
 * v_wind = 0 keeps the inertial frame (|p| kept).  Not supported with the
 * network field source (GC_EINVAL from gc_advance).
 * Ensemble parameters (q, m, lambda_par, r_in, r_out, max_steps, drift_free,
 * scatter_law, seed) are stored per ensemble index; injecting again into an
 * existing ensemble index replaces them.  lambda_par <= 0 disables scattering;
 * max_steps > 0 makes a particle FINISHED after that many steps; drift_free = 1
 * keeps only v_par b in dR/dt (Sect. 3.2); scatter_law 0: mu' = 1 - 2a (Eq. 10),
 * 1: mu' = +-sqrt(a) (Eq. 12).
 * Errors: GC_ESTATE before gc_load_field; GC_EINVAL for ensemble >= 4096,
 * m <= 0, q == 0, ekin <= 0, r_in >= r_out, mu_lo/mu_hi outside [-1, 1],
 * rebirth_steps > 2^24, v_wind outside [0, 0.1 c).  n == 0 is a no-op. */
typedef struct {
    uint32_t ensemble;
    uint32_t first_id;
    uint64_t n;
    uint64_t seed;
    double q, m;            /* C, kg */
    double ekin;            /* J */
    double r0, lat0, lon0;  /* m, rad, rad */
    double dlon, dr0, dlat; /* half-widths */
    double mu_lo, mu_hi;
    double lambda_par;      /* m */
    double r_in, r_out;     /* m */
    int64_t max_steps;
    int32_t drift_free;
    int32_t scatter_law;
    int64_t rebirth_steps;  /* > 0: rebirth of particles that exit before this step count */
    double v_wind;          /* m/s; > 0: scattering centres move with a radial wind (Sect. 3.3) */
} gc_inject_desc;

gc_status gc_inject(gc_ctx *ctx, const gc_inject_desc *desc);

/* ------------------------------------------------------------- advance */
/* Advance every active particle by n_steps steps of size dt (s), or until it
 * exits, finishes or meets a non-finite value.  Per step (Eqs. 5-6 and 9-10):
 * gather at X^n; apply a pending collision; F^n; bootstrap F^{n-1} if flagged;
 * predictor X*; gather and F*; corrector X^{n+1}; path += (|v_par^n| + |v_par*|) dt / 2,
 * collision pending once the path reaches the free path; exit test (with
 * rebirth when the ensemble asks for it); finish test.
 * tau = dt / (previous dt) on the first step after a change of dt.
 * The work is split in launches of chunk_steps steps, each preceded by the
 * configured reordering.  Host waits: with tail_threshold > 0 the call waits,
 * after queueing each chunk, for the chunk queued 3 chunks before it (so a
 * call returns with at most 3 chunks still running); with tail_threshold = 0
 * it returns without waiting.  Errors: GC_ESTATE without field; GC_EINVAL if
 * dt is not finite and > 0 or n_steps < 0. */
gc_status gc_advance(gc_ctx *ctx, double dt, int64_t n_steps);

/* Same work as gc_advance, captured once per (dt, n_steps, options) into a
 * hipGraph and replayed on later calls with identical arguments.  In the graph
 * every chunk reorders and runs the push the options select (the persistent
 * push picks its tail forms on the device).  With tail_threshold > 0 the call
 * keeps the host at most 3 calls ahead of the device (it waits for the replay
 * issued 3 calls earlier), and once the live count read back is below
 * tail_threshold it runs the chunks eagerly with the tail policy, as
 * gc_advance, instead of replaying; results are bitwise the same either way.
 * With tail_threshold = 0 it always replays and never waits. */
gc_status gc_advance_graph(gc_ctx *ctx, double dt, int64_t n_steps);

/* -------------------------------------------------------------- moments */
/* Snapshot statistics (Sect. 3: <sin^2 alpha>(r), energy versus age near
 * 1 AU, pitch-cosine distributions).  out: caller-owned DEVICE buffer of
 * gc_moments_size(spec) int64 values, overwritten (accumulate == 0) or added
 * to (accumulate != 0: the sum over snapshots of the steady-state statistics
 * of Sect. 3, one call per snapshot, no host round trip):
 *   [0..3] particles per status, [4] sum of collision counts, [5] sum of steps,
 *   [6] sum over active particles of floor(r/len_unit * 2^32),
 *   [7] active particles with at least one collision,
 *   then n_rbins x {count, sum floor(sin^2 alpha * 2^32), sum floor(E/e_unit * 2^16)}
 *     for active particles with r in [r_lo, r_hi),
 *   then n_mubins counts of mu = cos(alpha) on [-1, 1] for active particles with
 *     r in [sel_r_lo, sel_r_hi), age in [age_lo, age_hi), k >= min_collisions,
 *   then n_agebins x n_ebins counts of (age on [0, age_max), E on [e_lo, e_hi))
 *     for active particles with r in [sel_r_lo, sel_r_hi).
 * The three binned sections count only particles whose current generation
 * began at a step count >= min_birth (Sect. 3 keeps particles injected once
 * the steady state is reached); [0..7] count every particle.
 * alpha is the pitch angle, E = (gamma - 1) m c^2 with |B| interpolated at the
 * particle, age = time since (re)injection.  Integer sums: the result does not
 * depend on the particle order.  Errors: GC_EINVAL for out == NULL, negative
 * bin counts, empty ranges, or more than 8192 outputs. */
typedef struct {
    int32_t n_rbins;   double r_lo, r_hi;
    int32_t n_mubins;
    double sel_r_lo, sel_r_hi;
    double age_lo, age_hi;
    int32_t min_collisions;
    int32_t n_agebins; double age_max;
    int32_t n_ebins;   double e_lo, e_hi;
    double e_unit;     /* J per energy unit */
    double len_unit;   /* m per length unit */
    uint32_t min_birth;  /* binned sections: generation began at step count >= min_birth */
    int32_t accumulate;  /* nonzero: add into out instead of overwriting it */
} gc_moment_spec;

int64_t gc_moments_size(const gc_moment_spec *spec);
gc_status gc_moments(gc_ctx *ctx, const gc_moment_spec *spec, int64_t *out);

/* --------------------------------------------------- state checkpointing */
/* Per-particle state in global injection order (index g = order of injection).
 * Every pointer is a caller-owned DEVICE array of n entries; NULL members are
 * skipped.  mu is mu_B / m (m^2 s^-2 T^-1).  (cr, cth, cph, cu, ct) are the
 * Kahan compensation terms of the FP32 form (zero otherwise). */
typedef struct {
    double *r, *th, *ph, *u, *mu;
    double *fr, *fth, *fph, *fu;       /* F^{n-1} */
    double *dtp, *s, *ell, *t;
    double *cr, *cth, *cph, *cu, *ct;
    uint32_t *k, *flags, *status, *step, *id, *ens;
    uint32_t *birth;                   /* step count at which the current generation began */
} gc_state_view;

/* Number of particles injected so far. */
gc_status gc_count(const gc_ctx *ctx, uint64_t *n);
/* Copy the state out (async). */
gc_status gc_get_state(gc_ctx *ctx, const gc_state_view *dst);
/* Replace the whole state by n particles read from src (async); every member
 * must be non-NULL.  ens values must name ensembles already injected. */
gc_status gc_set_state(gc_ctx *ctx, const gc_state_view *src, uint64_t n);
/* Copy the collision log out (async): dst is a DEVICE array of n x log_depth
 * uint32, entry [g][k] = step count at which collision k+1 of particle g was
 * applied, 0xFFFFFFFF if none.  GC_ESTATE if log_depth is 0. */
gc_status gc_get_log(gc_ctx *ctx, uint32_t *dst);

/* Slot order of the particles after the last reorder (the cell binning of the
 * trilinear gathers' locality, Sect. 2.2): every pointer is a caller-owned
 * DEVICE buffer or NULL (skipped).  slot_gid: gc_count() uint32, the global
 * injection index of the particle in each slot.  slot_key: gc_count() uint32,
 * the cell key the last reorder sorted that slot on (GC_ORDER_BIN only; with
 * c = bin_coarsen, key = ((i >> c) nth_c + (j >> c)) nph_c + (k >> c) for the
 * lower stencil node (i, j, k) of the particle's position, nth_c and nph_c the
 * coarsened node counts; inactive particles, and every slot past the prefix
 * that reorder sorted, get nr_c nth_c nph_c).  n_live: one uint32, the
 * number of particles that were active at that reorder (they fill the slots
 * below it).  Async.  The push moves particles between reorders and the tail
 * policy skips reorders, so the keys describe the positions of the last
 * reorder, not the current ones.  Errors: GC_EINVAL if every pointer is NULL;
 * GC_ESTATE if no reorder ran since the last gc_inject, gc_set_state or
 * growth of the state, or if slot_key is given and the last reorder was not a
 * cell binning. */
gc_status gc_get_order(gc_ctx *ctx, uint32_t *slot_gid, uint32_t *slot_key, uint32_t *n_live);

/* ----------------------------------------------------------- counters */
/* Waits for the stream.  push_ms: summed duration of push launches recorded
 * with timing = 1 or 2; n_push: their number; reorder_ms, n_reorder: the same for
 * reorders (their kernels from the first to the last, less any push between),
 * with timing = 1; particle_steps: steps taken by active
 * particles since the context was created or counters were reset.  form_*: the
 * same split by form of the grid push: [0] throughput form (and the
 * neural-field push), [1] all loads of a gather in flight, [2] four lanes per
 * particle (tail_threshold).  The persistent push splits its steps by form the
 * same way (the device picks the form from the live count) and books the time
 * of its launches under [0].  GC_EDEVICE if a cell-binning sort pass recorded
 * that it stopped waiting for an earlier tile (bounded wait; not expected on
 * working hardware): the particle order, and so the run, is then invalid
 * until gc_set_state loads a state again. */
typedef struct {
    double push_ms;
    int64_t n_push;
    double reorder_ms;
    int64_t n_reorder;
    uint64_t particle_steps;
    double form_ms[3];
    int64_t form_launches[3];
    uint64_t form_steps[3];
} gc_counters;
gc_status gc_get_counters(gc_ctx *ctx, gc_counters *out);
gc_status gc_reset_counters(gc_ctx *ctx);

/* --------------------------------------------------------- neural field */
/* A Fourier-feature network that can replace the gridded field in the push
 * (field_source = GC_SOURCE_MLP); the grid stays loaded as fallback and judge
 * (injection, binning and moments keep using it).  With x = ((r - r_min) /
 * (r_max - r_min), th/pi) of the loaded grid:
 *   psi_j = 2 pi (a_j x_0 + b_j x_1) + n_j ph  (j < 64, n_j integer),
 *   h0 = [sin psi_0, cos psi_0, sin psi_1, ...]  (128 features),
 *   h_l = silu(W_l h_{l-1} + c_l) for l = 1..6 (W_l 128 x 128),
 *   y = W_o h_6 + c_o (6 outputs),
 *   B_i = S_i (r_ref/r)^p_i y_i, E_i = S_{i+3} (r_ref/r)^p_{i+3} y_{i+3};
 * grad|B| and (b.grad)b from the derivatives of B along (r, th, ph), carried
 * forward through the network (three tangents).  Products run in BF16 on the
 * matrix cores with FP32 accumulation; parameters are kept in FP32. */
#define GC_MLP_PARAMS 99846   /* W[6][128][128] | c[6][128] | W_o[6][128] | c_o[6], FP32 */

typedef struct {
    double freq[64][3];       /* a_j, b_j, n_j */
    double r_ref;             /* m */
    double scale[6];          /* S_c */
    double power[6];          /* p_c */
    const float *params;      /* HOST pointer to GC_MLP_PARAMS values (copied), NULL: all zero */
} gc_mlp_desc;

/* Install (or replace) the network; resets the optimizer state.  Waits.
 * Errors: GC_ESTATE before gc_load_field (the input normalization uses its
 * radial range); GC_EINVAL for non-integer n_j or non-finite values. */
gc_status gc_mlp_set(gc_ctx *ctx, const gc_mlp_desc *desc);
/* Copy the FP32 parameters (GC_MLP_PARAMS floats, HOST) out.  Waits. */
gc_status gc_mlp_get_params(gc_ctx *ctx, float *host_out);
/* Copy the gradient of the last gc_mlp_train_step out (HOST).  Waits. */
gc_status gc_mlp_get_grads(gc_ctx *ctx, float *host_out);

typedef struct {
    double lr, beta1, beta2, eps;   /* Adam */
    double wc[6];                   /* weights of the six normalized outputs in the loss */
    double beta_pair;               /* weight of the paired-difference term */
    int32_t step;                   /* Adam step number (>= 1) */
    int32_t apply;                  /* 0: compute loss and gradient only */
} gc_mlp_train_opts;

/* One training step on n_pairs paired points.  pts: DEVICE array of 3 x (2 n)
 * doubles (r[2n], then th[2n], then ph[2n]); point n_pairs + i is the partner
 * of point i.  tgt: DEVICE array of (2 n) x 6 doubles, the field (B, E) to fit
 * at every point.  Loss (normalized outputs y, targets t = tgt / envelope):
 *   L = (1/n) sum_i sum_c w_c [(y_c(x_i) - t_c(x_i))^2
 *        + beta ((y_c(x'_i) - y_c(x_i)) - (t_c(x'_i) - t_c(x_i)))^2].
 * *loss (HOST) receives L.  Waits. */
gc_status gc_mlp_train_step(gc_ctx *ctx, const double *pts, const double *tgt, int64_t n_pairs,
                            const gc_mlp_train_opts *opts, double *loss);

/* gc_mlp_train_step for callers that cannot allocate device memory (code under
 * HIP graph capture around the device work, serving or training loops, or
 * harnesses that forbid allocation): the same step, bitwise the same loss,
 * gradient and update, with its training workspace (activations,
 * pre-activations, output gradients, split-K and column-sum partials, loss
 * partials) in a static device array of the library instead of memory the
 * context allocates.  The array holds 24.2 MiB, enough for n_pairs <= 2048,
 * and each device the library runs on keeps its own copy until the process
 * ends.  The call allocates nothing (no hipMalloc, hipFree or allocator
 * callback); it reads the loss back and waits, like gc_mlp_train_step.
 * Every call on one device shares that device's array: calls that overlap on
 * one device (two contexts on different streams, or two host threads) race,
 * and the array keeps the last call's contents.  Errors: as gc_mlp_train_step,
 * and GC_EINVAL for n_pairs > 2048; GC_EDEVICE if the array's device address
 * could not be read when the context was created. */
gc_status gc_mlp_train_step_noalloc(gc_ctx *ctx, const double *pts, const double *tgt, int64_t n_pairs,
                                    const gc_mlp_train_opts *opts, double *loss);

/* Field at n points (DEVICE pts: r[n], th[n], ph[n]; DEVICE out: n x 12, the
 * components in the order of the grid): gc_mlp_eval from the network,
 * gc_field_sample by trilinear interpolation of the loaded grid.  Async. */
gc_status gc_mlp_eval(gc_ctx *ctx, const double *pts, int64_t n, double *out);
gc_status gc_field_sample(gc_ctx *ctx, const double *pts, int64_t n, double *out);

/* ------------------------------------------------------------ autotuner */
/* Choose launch parameters by timing the context's own workload: coordinate
 * descent over workgroup size, then bin coarsening, then steps per chunk,
 * then persistent-form tile sizes.  Candidates keep the form (grid or
 * persistent) the context has on entry, except the tile candidates, which
 * are always persistent.  Each candidate starts from the
 * same saved state and runs probe_steps steps of size dt, timed with HIP
 * events; the state is restored afterwards, so the particles do not advance.
 * Candidate lists with n_* = 0 keep the current value.  The best options are
 * applied to the context and returned with their rate (active particle-steps
 * per second).  Waits for the stream.  Errors: GC_ESTATE without field or
 * particles; GC_EINVAL for probe_steps < 1 or invalid candidates. */
typedef struct {
    int32_t n_block;   int32_t block[3];
    int32_t n_coarsen; int32_t coarsen[4];
    int32_t n_chunk;   int32_t chunk[6];
    int32_t n_tile;    int32_t tile[4];     /* persistent-form tiles (0 candidates: grid form only) */
    int64_t probe_steps;
    double dt;
} gc_tune_space;

typedef struct {
    gc_options best;
    double best_rate;        /* particle-steps/s of the best candidate */
    double default_rate;     /* ... of the options the context had on entry */
    int32_t n_tried;
    int32_t pad;
} gc_tune_result;

gc_status gc_autotune(gc_ctx *ctx, const gc_tune_space *space, gc_tune_result *out);

/* Copy n_bytes from src to dst (both device) with a plain streaming kernel;
 * used to calibrate hardware traffic counters against a known byte count. */
gc_status gc_copy_probe(gc_ctx *ctx, void *dst, const void *src, uint64_t n_bytes);

/* Gather ceiling of the push (the denominator of its roofline): every particle
 * in the live prefix of the last reorder makes the push's two trilinear
 * gathers per step for n_steps steps while moving on the straight line
 * X + k dt F^{n-1}, with the push's layout, slot order and launch shape but
 * none of its arithmetic.  sink: DEVICE array of at least gc_count() doubles
 * (receives a checksum per slot).  The particle state is not modified; the
 * probe's particle-steps are added to the particle_steps counter.  Async.
 * Errors: GC_ESTATE without a field; GC_EINVAL for dt <= 0 or n_steps < 0. */
gc_status gc_gather_probe(gc_ctx *ctx, double dt, int32_t n_steps, double *sink);

#ifdef __cplusplus
}
#endif
#endif /* GCPUSH_H */
