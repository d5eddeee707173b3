// gc_step.h -- pieces of the guiding-centre step shared by the push kernels
// (grid field source in gc_push.hip, neural field in gc_push_mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "gc_device.h"
#include "gc_internal.h"

namespace gc {

template <int PREC> struct PrecT;
template <> struct PrecT<GC_PREC_F64> { using R = double; using A = double; static constexpr bool kKahan = false; };
template <> struct PrecT<GC_PREC_F32_ACC64> { using R = float; using A = double; static constexpr bool kKahan = false; };
template <> struct PrecT<GC_PREC_F32_KAHAN> { using R = float; using A = float; static constexpr bool kKahan = true; };

// x += d with Kahan compensation c (true sum ~ x - c)
template <typename A>
__device__ __forceinline__ void kahan_add(A &x, A &c, A d) {
    A y = d - c;
    A t = x + y;
    c = (t - x) - y;
    x = t;
}

// Generator block of collision k1 of generation gen (counter (id, k1, 0, gen),
// key (seed, ensemble)): new pitch cosine from a1 (Eq. 10, or Eq. 12 with the
// sign from a2) and the next free path -lambda ln(1 - a0).  Kept out of line:
// it runs for a few steps in a thousand, and inlined it would raise the push's
// register count.
struct CollisionDraw { double mun, ell; };

__device__ __noinline__ CollisionDraw draw_collision(uint32_t pid, uint32_t k1, uint32_t gen, uint64_t seed,
                                                     uint32_t ens, int law, double lambda) {
    const U64x4 rb = philox4x64_10(pid, k1, kPurposePath, gen, seed, ens);
    const double a0 = u01(rb.v[0]), a1 = u01(rb.v[1]), a2 = u01(rb.v[2]);
    CollisionDraw d;
    d.mun = law == 1 ? (a2 < 0.5 ? -1.0 : 1.0) * sqrt(a1) : 1.0 - 2.0 * a1;
    d.ell = -lambda * log(1.0 - a0);
    return d;
}

// Initial state of particle pid (Sect. 3 injection), FP64: site, spreads and
// pitch cosine from block (pid, 0, inject, 0), the same for every generation;
// the first free path of generation gen from block (pid, 0, path, gen);
// mu_B / m from |B| interpolated at the site.  status is EXITED for a site
// outside the shell, NONFINITE for a non-finite field there.
struct BirthState {
    double r, th, ph, u, mu, ell;
    uint32_t status;
};

template <int FDT>
__device__ __forceinline__ BirthState birth_state(const FieldDev &f, const EnsDev &e, uint32_t pid, uint32_t gen) {
    const U64x4 a = philox4x64_10(pid, 0, kPurposeInject, 0, e.seed, e.ensemble);
    BirthState b;
    b.ph = e.lon0 + e.dlon * (2.0 * u01(a.v[0]) - 1.0);
    const double mup = e.mu_lo + (e.mu_hi - e.mu_lo) * u01(a.v[1]);
    b.r = e.r0 + e.dr0 * (2.0 * u01(a.v[2]) - 1.0);
    const double lat = e.lat0 + e.dlat * (2.0 * u01(a.v[3]) - 1.0);
    b.th = 0.5 * kPi - lat;
    const double gamma = 1.0 + e.ekin / (e.m * kC * kC);
    const double pm = kC * sqrt(gamma * gamma - 1.0);        // |p| / m
    b.u = pm * mup;
    const U64x4 c = philox4x64_10(pid, 0, kPurposePath, gen, e.seed, e.ensemble);
    b.ell = e.lambda > 0.0 ? -e.lambda * log(1.0 - u01(c.v[0])) : __builtin_inf();
    b.status = GC_ACTIVE;
    b.mu = 0.0;
    if (b.r < e.r_in || b.r > e.r_out || b.th < f.th_lo || b.th > f.th_hi) {
        b.status = GC_EXITED;
    } else {
        // the gather of the push, one node pair in registers at a time (this
        // runs out of line, and its register count bounds the caller's)
        double g[12];
        GatherPlan<double> gp;
        bool ok = gather_plan(f, b.r, b.th, b.ph, gp);
        if (ok) {
#pragma unroll
            for (int c = 0; c < 12; ++c) g[c] = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                Pair<FDT> p;
                p.load(f.data, gp.off[q]);
                gather_add<FDT, double>(f, gp, q, p, g);
                __builtin_amdgcn_sched_barrier(0);
            }
            ok = finite12(g);
        }
        if (!ok) b.status = GC_NONFINITE;
        else b.mu = pm * pm * (1.0 - mup * mup) / (2.0 * sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]));
    }
    return b;
}

// Rebirth inside a push kernel: out of line (it runs once per exit), reading
// the field description and the ensemble from device memory.
template <int FDT>
__device__ __noinline__ BirthState rebirth_state(const FieldDev *f, const EnsDev *e, uint32_t pid, uint32_t gen) {
    return birth_state<FDT>(*f, *e, pid, gen);
}

__device__ __forceinline__ void count_steps(const PushArgs &a, uint32_t taken) {
    // one atomic per wavefront
    uint32_t v = taken;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(a.steps_done, (unsigned long long)v);
}

}  // namespace gc
