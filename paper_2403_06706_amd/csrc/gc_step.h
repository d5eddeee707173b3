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

// Collision in the frame of the scattering centres when they move with a
// radial wind of speed vw (Sect. 3.3).  The wind's component across B is the
// E x B drift the guiding centre already moves with; along b it is
// V = vw b_r.  A Lorentz boost along b by V takes (p_par, energy) to the wind
// frame (p_perp unchanged); the collision keeps |p~| and sets
// p~_par = mun |p~|; the boost back gives the new u = p_par / m.  In: u, mu =
// mu_B / m, |B|, B_r, mun.  Out: u_new and (|p~| / m)^2, from which the
// caller takes mu_B / m = |p~|^2 (1 - mun^2) / (2 |B|).
template <typename R>
__device__ __forceinline__ void wind_collision(R u, R mu, R B, R Br, R vw, R mun, R &u_new, R &P2) {
    const R V = vw * Br / B;
    const R G = rsqrt_nr((R)1 - V * V * (R)kInvC2);
    const R pp2 = (R)2 * mu * B;                       // (p_perp / m)^2
    const R gam = sqrt((R)1 + (u * u + pp2) * (R)kInvC2);
    const R uw = G * (u - V * gam);                    // wind frame: p_par / m
    const R gw = G * (gam - V * u * (R)kInvC2);        // wind frame: gamma
    P2 = uw * uw + pp2;
    u_new = G * (mun * sqrt(P2) + V * gw);
}

// Speed along b against the scattering centres, for the path of Eq. 9:
// |v_par| for centres at rest, Gamma |v_par - V| for centres moving with the
// wind (V = vw b_r; a boost along b turns dx - V dt into Gamma (v_par - V) dt).
template <typename R>
__device__ __forceinline__ R path_speed(R vp, const R g[12], R vw) {
    if (!(vw > (R)0)) return fabs(vp);
    const R V = vw * g[0] * rsqrt_nr(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    return rsqrt_nr((R)1 - V * V * (R)kInvC2) * fabs(vp - V);
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
        bool ok = gather_plan<FDT>(f, b.r, b.th, b.ph, gp);
        if (ok) {
#pragma unroll
            for (int c = 0; c < 12; ++c) g[c] = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                Pair<FDT> p;
                p.load(f.data, gp.off[q], gp.dk, gp.cs);
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

__device__ __forceinline__ void count_steps(unsigned long long *counter, uint32_t taken) {
    // one atomic per wavefront
    uint32_t v = taken;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(counter, (unsigned long long)v);
}
__device__ __forceinline__ void count_steps(const PushArgs &a, uint32_t taken) { count_steps(a.steps_done, taken); }

}  // namespace gc
