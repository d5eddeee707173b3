// gc_internal.h -- structures shared by the host library and its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcpush.h"

namespace gc {

constexpr int kMaxEnsembles = 4096;
constexpr int kMaxMoments = 8192;
constexpr int64_t kMaxRebirthSteps = 1 << 24;   // generations fit the 24 flag bits above GC_FLAG_GEN_SHIFT
constexpr int kNumComp = 12;

// Per-ensemble parameters, indexed by the particle's ensemble field.
struct EnsDev {
    double qm;          // q / m (C/kg)
    double iqm;         // m / q
    double m;           // kg
    double lambda;      // mean free path (m); <= 0: no scattering
    double r_in, r_out; // exit shell (m)
    uint64_t seed;      // generator key word 0
    int64_t max_steps;  // > 0: FINISHED after this many steps
    uint32_t ensemble;  // generator key word 1
    int32_t drift_free;
    int32_t scatter_law;
    int32_t pad;
    // injection site and spreads (Sect. 3), read again when a particle is reborn
    double ekin, r0, lat0, lon0, dlon, dr0, dlat, mu_lo, mu_hi;
    int64_t rebirth_steps;  // an exit at a step count below this is followed by a rebirth
    double v_wind;          // > 0: scattering centres move with a radial wind of this speed (m/s)
};

// Packed field on the device: [nr][nth][nph+1][12], the extra phi node repeats
// node 0 so that every phi pair (k, k+1) is contiguous.
struct FieldDev {
    const void *data;
    int32_t nr, nth, nph, dtype;
    double r_min;
    double inv_dr, inv_dth, inv_dph, inv_nph;
    double th_lo, th_hi;  // first and last theta node (exit bounds)
    float scale[12];      // GC_F16: stored value * scale = field value
};

// Structure-of-arrays particle state (one slot per particle).
struct SoA {
    double *r, *th, *ph, *u, *mu;
    double *fr, *fth, *fph, *fu;
    double *dtp, *s, *ell, *t;
    double *cr, *cth, *cph, *cu, *ct;
    uint32_t *k, *flags, *status, *step, *id, *ens, *gid, *birth;
};
constexpr int kNumDoubleArrays = 18;
constexpr int kNumU32Arrays = 8;

struct PushArgs {
    SoA st;
    FieldDev f;
    FieldDev fx;                   // full Eqs. 1-2: the extra node array (mode 2)
    const FieldDev *fdev;          // device copy of f (for the out-of-line rebirth)
    const EnsDev *ens;
    const uint32_t *n_active;      // device count of slots to visit
    uint32_t n_slots;              // grid coverage
    int32_t n_steps;
    double dt;
    unsigned long long *steps_done;
    uint32_t *log;                 // [n_total][log_depth] indexed by gid
    int32_t log_depth;
    int32_t tile;                  // persistent mode: particles per work item
    uint32_t *queue;               // persistent mode: next tile counter
    int32_t mode;                  // 0 plain, 1 rebirth or wind-frame scattering, 2 also the full Eqs. 1-2
};

}  // namespace gc
