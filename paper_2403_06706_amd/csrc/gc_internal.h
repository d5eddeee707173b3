// gc_internal.h -- structures shared by the host library and its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcpush.h"

namespace gc {

constexpr int kMaxEnsembles = 4096;
// Tail policy: below tail_threshold / kQuadShare live particles the push takes
// the four-lanes-per-particle form (above it, in the tail, all pairs in flight).
constexpr uint32_t kQuadShare = 4;
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

// Packed field on the device.  nph + 1 phi nodes (the last repeats node 0, so
// a phi pair (k, k+1) needs no wrap).  The 12 components of a node are cut in
// nch chunks of W consecutive components, one load each (16 bytes for FP32
// and FP64, 8 for FP16).  Nodes are grouped in blocks of 4 (r) x 2 (phi);
// one chunk of a block's 8 nodes is contiguous (one 128-byte line for FP32
// and FP64), and blocks follow one another along r, then the chunk index,
// then phi, then theta.  Chunk c of node (i, j, k) is at element
//   gI(i) + gK(k) + gJ(j) + c cs,
//   gI(i) = (i >> 2) 8 W + (i & 3) W,
//   gK(k) = (k >> 1) ks + (k & 1) 4 W,   ks = nch cs,
//   gJ(j) = j js,                        js = nK ks,
// with cs = nI 8 W, nI = ceil(nr / 4), nK = ceil((nph + 1) / 2); padding
// nodes hold zeros.  A cell-sorted wavefront spreads along the field, mostly
// in r and phi; in this order lanes at nearby nodes share the cache line of
// each load.
constexpr uint32_t kLayBr = 4, kLayBk = 2, kLayB = kLayBr * kLayBk;   // nodes per block (r, phi)

struct FieldLayout {
    uint32_t W, nch;      // components per chunk, chunks per node
    uint32_t cs, ks, js;  // element strides: chunk, phi block, theta row
    uint64_t total;       // elements, padding included
};

__host__ __device__ inline FieldLayout field_layout(int nr, int nth, int nph, int dtype) {
    FieldLayout L;
    L.W = dtype == GC_F64 ? 2u : 4u;
    L.nch = 12u / L.W;
    const uint32_t nI = ((uint32_t)nr + kLayBr - 1) / kLayBr, nK = ((uint32_t)nph + 1 + kLayBk - 1) / kLayBk;
    L.cs = nI * kLayB * L.W;
    L.ks = L.nch * L.cs;
    L.js = nK * L.ks;
    L.total = (uint64_t)nth * L.js;
    return L;
}

struct FieldDev {
    const void *data;
    int32_t nr, nth, nph, dtype;
    double r_min;
    double inv_dr, inv_dth, inv_dph, inv_nph;
    double th_lo, th_hi;  // first and last theta node (exit bounds)
    float scale[12];      // GC_F16: stored value * scale = field value
    uint32_t cs, ks, js;  // layout strides (field_layout)
    // Node records of the same values, [nr][nth][nph+1][12] of the storage
    // type, for the four-lanes-per-particle form of FP32 and FP64 fields (its
    // lanes take three components of a node each); NULL otherwise.
    const void *rec;
    // Nonzero when every value of the grid is finite and at most kTameField
    // in magnitude: then a trilinear combination of its nodes (weights in
    // [0, 1]) and the sum of twelve such cannot overflow, in FP32 or FP64, and
    // the push kernels (an instantiation of their own) and the gather probe
    // skip the test of a gather's result for non-finite values.
    int32_t tame;
};
constexpr double kTameField = 1e30;

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
    SoA st;                        // the state written
    SoA src;                       // the state read: st itself, or with perm the other buffer
    const uint32_t *perm;          // null, or a reorder's permutation that the push applies: the
                                   // particle of slot i is read from src at perm[i] and every
                                   // field of it written to st at i
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
    uint32_t tail;                 // persistent mode: tail threshold of the live count (0: throughput form only)
    int32_t mode;                  // 0 plain, 1 rebirth or wind-frame scattering, 2 also the full Eqs. 1-2
};

}  // namespace gc
