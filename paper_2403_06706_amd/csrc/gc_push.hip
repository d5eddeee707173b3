// gc_push.hip -- the hot path: advance particles by a chunk of steps.
//
// One particle per lane.  Its state is loaded into registers once per launch,
// advanced for n_steps steps of the third-order predictor-corrector (Eqs. 5-6)
// with hard-sphere scattering (Eqs. 9-10), and stored once.  Each step makes
// two trilinear gathers of the 12 field components (at X^n and at X*), a third
// one on bootstrap steps (injection and after a collision).
#include <hip/hip_runtime.h>

#include "gc_device.h"
#include "gc_launch.h"
#include "gc_step.h"

namespace gc {

// Forms of the push (all bitwise identical in their results):
//   kFormThroughput  one lane per particle, two node pairs of a gather in registers at a time;
//   kFormAllPairs    one lane per particle, all four pairs of a gather in flight;
//   kFormQuad        four lanes per particle (an aligned quad): each lane interpolates three
//                    of the twelve components of every gather (FP16 fields: loads one node
//                    pair), the quad shares the results, all four run the rest of the step
//                    on identical values, lane gl = 0 writes.
enum { kFormThroughput = 0, kFormAllPairs = 1, kFormQuad = 2 };

// MODE 0: the reduced equations, no rebirth, centres at rest.  MODE 1: also
// rebirth and scattering in the wind frame (Sect. 3 and 3.3); a separate
// instantiation because the out-of-line rebirth raises the register count of
// the FP32 forms.  MODE 2: also the full Eqs. 1-2 (the extra node array is
// gathered with the field's stencil at each evaluation; no quad form).
// TAME: the field is tame (FieldDev::tame), so the gathers skip their
// finiteness test (compiled out; a run-time branch around it measured slower,
// and in the quad form no faster than the test).
template <int PREC, int FDT, int MODE, int FORM = kFormThroughput, bool TAME = false>
__device__ __forceinline__ uint32_t advance_slot(const PushArgs &a, uint32_t slot, uint32_t gl = 0) {
    constexpr bool EXT = MODE >= 1;
    constexpr bool FULL = MODE == 2;
    using R = typename PrecT<PREC>::R;
    using A = typename PrecT<PREC>::A;
    constexpr bool kKahan = PrecT<PREC>::kKahan;
    // The particle of this slot is read from sr at ls and written to st at
    // slot: the same place, or (a reorder's permutation applied by the push)
    // its place in the other state buffer.  In place, a stopped particle costs
    // one load.  Moved, every field is loaded at once, one round trip after
    // the permutation's.
    const SoA &st = a.st, &sr = a.src;
    const bool moved = a.perm != nullptr;
    const uint32_t ls = moved ? a.perm[slot] : slot;
    if (!moved && sr.status[ls] != GC_ACTIVE) return 0;
    uint32_t status = sr.status[ls], flags = sr.flags[ls], k = sr.k[ls], step = sr.step[ls];
    const uint32_t ens_raw = sr.ens[ls], pid = sr.id[ls];
    const uint32_t gid = sr.gid[ls], birth0 = sr.birth[ls];
    double r0 = sr.r[ls], th0 = sr.th[ls], ph0 = sr.ph[ls], u0 = sr.u[ls], t0 = sr.t[ls];
    double fr0 = sr.fr[ls], fth0 = sr.fth[ls], fph0 = sr.fph[ls], fu0 = sr.fu[ls];
    double mu0 = sr.mu[ls], dtp0 = sr.dtp[ls], s0 = sr.s[ls], ell0 = sr.ell[ls];
    double cr0 = 0, cth0 = 0, cph0 = 0, cu0 = 0, ct0 = 0;
    if (kKahan) { cr0 = sr.cr[ls]; cth0 = sr.cth[ls]; cph0 = sr.cph[ls]; cu0 = sr.cu[ls]; ct0 = sr.ct[ls]; }
    // The empty statements below take every loaded value, so the loads are all
    // issued before the status test (else the compiler issues the status load
    // alone, and the others after its round trip).
#define GC_LOADED(x) asm volatile("" : "+v"(x))
    GC_LOADED(status); GC_LOADED(flags); GC_LOADED(k); GC_LOADED(step);
    GC_LOADED(r0); GC_LOADED(th0); GC_LOADED(ph0); GC_LOADED(u0); GC_LOADED(t0);
    GC_LOADED(fr0); GC_LOADED(fth0); GC_LOADED(fph0); GC_LOADED(fu0);
    GC_LOADED(mu0); GC_LOADED(dtp0); GC_LOADED(s0); GC_LOADED(ell0);
    if (kKahan) { GC_LOADED(cr0); GC_LOADED(cth0); GC_LOADED(cph0); GC_LOADED(cu0); GC_LOADED(ct0); }
#undef GC_LOADED
    // (moved: every slot is active, a reorder puts the active particles first)
    if (status != GC_ACTIVE) return 0;
    const uint32_t step0 = step;
    const uint32_t eidx = min(ens_raw, (uint32_t)(kMaxEnsembles - 1));
    const EnsDev e = a.ens[eidx];
    uint32_t birth = 0;
    bool reborn = false;
    A X0 = (A)r0, X1 = (A)th0, X2 = (A)ph0, X3 = (A)u0;
    A T = (A)t0;
    A c0 = (A)cr0, c1 = (A)cth0, c2 = (A)cph0, c3 = (A)cu0, cT = (A)ct0;
    R fp0 = (R)fr0, fp1 = (R)fth0, fp2 = (R)fph0, fp3 = (R)fu0;
    R mu = (R)mu0, dtp = (R)dtp0, s = (R)s0, ell = (R)ell0;
    const R qm = (R)e.qm, iqm = (R)e.iqm;
    const bool drift_free = e.drift_free != 0;
    const bool scatter = e.lambda > 0.0;
    const R vw = EXT ? (R)e.v_wind : (R)0;          // > 0: scattering centres move with the wind
    const R h = (R)a.dt;
    const double r_in = e.r_in, r_out = e.r_out, th_lo = a.f.th_lo, th_hi = a.f.th_hi;

    for (int it = 0; it < a.n_steps; ++it) {
        // Field evaluations of the step: at X^n, at X^{n-1} = X^n - dt F^n on
        // bootstrap steps only, and at the predictor X*.
        R Fn[4], Fs[4], vpn = 0, vps = 0, tau = 1;
        // A pending collision k+1 draws its generator block before the first
        // gather of the step (few live registers here); it is applied once the
        // gather at X^n gives |B| there.
        R mun = 0, ell_new = 0;
        if (flags & GC_FLAG_PENDING) {
            const CollisionDraw d = draw_collision(pid, k + 1, flags >> GC_FLAG_GEN_SHIFT, e.seed, e.ensemble,
                                                   e.scatter_law, e.lambda);
            mun = (R)d.mun;
            ell_new = (R)d.ell;
        }
        R px = (R)X0, pth = (R)X1, pph = (R)X2, pu = (R)X3;
        bool bad = false;
        // the gather at a point (xg: the extra node array, full equations only)
        auto gather_at = [&](R x, R t, R p, R g[12], R xg[12], bool &xok) -> bool {
            xok = true;
            if constexpr (FULL) return gather2<FDT, R, FORM == kFormAllPairs>(a.f, a.fx, x, t, p, g, xg, xok);
            else if constexpr (FORM == kFormQuad) return gather_quad<FDT, R, TAME>(a.f, x, t, p, gl, g);
            else return gather<FDT, R, FORM == kFormAllPairs, TAME>(a.f, x, t, p, g);
        };
        auto rhs_at = [&](R x, R t, R u, R g[12], R xg[12], R F[4], R &vp) {
            if constexpr (FULL) gc_rhs<R, true>(x, t, u, mu, qm, iqm, drift_free, g, F, vp, xg);
            else gc_rhs<R>(x, t, u, mu, qm, iqm, drift_free, g, F, vp);
        };
        // collision k+1 (Eqs. 9-10) at X^n: |p| kept, new pitch cosine and free path
        auto collide = [&](const R g[12]) {
            const R B = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            R p2 = pu * pu + (R)2 * mu * B;                  // (p/m)^2, kept in the inertial frame
            R un;
            if (EXT && vw > (R)0) wind_collision<R>(pu, mu, B, g[0], vw, mun, un, p2);
            else un = mun * sqrt(p2);
            X3 = (A)un;
            c3 = 0;
            pu = (R)X3;
            mu = p2 * ((R)1 - mun * mun) / ((R)2 * B);
            ell = ell_new;
            s = 0;
            k += 1;
            flags = (flags | GC_FLAG_BOOTSTRAP) & ~GC_FLAG_PENDING;
            if (a.log_depth > 0 && k <= (uint32_t)a.log_depth && gl == 0)
                a.log[(size_t)gid * a.log_depth + (k - 1)] = step;
        };
        // predictor, Eq. 5
        auto predict = [&]() {
            const R wn = (R)1 + (R)0.5 * tau, wq = (R)0.5 * tau;
            const R d0 = h * (wn * Fn[0] - wq * fp0), d1 = h * (wn * Fn[1] - wq * fp1);
            const R d2 = h * (wn * Fn[2] - wq * fp2), d3 = h * (wn * Fn[3] - wq * fp3);
            if (kKahan) {
                px = (R)(X0 + (d0 - c0)); pth = (R)(X1 + (d1 - c1)); pph = (R)(X2 + (d2 - c2)); pu = (R)(X3 + (d3 - c3));
            } else {
                px = (R)(X0 + (A)d0); pth = (R)(X1 + (A)d1); pph = (R)(X2 + (A)d2); pu = (R)(X3 + (A)d3);
            }
        };
        // One gather + right-hand side site that the stages loop through
        // (stage 0 at X^n, 1 at X^{n-1}, 2 at X*; lanes in different stages run
        // the same instructions) holds fewer registers than three sites in
        // straight-line code, which avoid the register copies between stages.
        // Either gives the same bits (multiply-adds are contracted only within
        // a source expression).  Three sites where measured faster (the
        // throughput and quad forms on FP32 fields, reduced equations); the
        // loop for all pairs of a gather in flight (slower with three sites)
        // and where three sites spill (full equations, FP64 and FP16 fields).
        constexpr bool kLoopSites = FORM == kFormAllPairs || FULL || FDT != GC_F32;
        if constexpr (kLoopSites) {
            int stage = 0;
            for (;;) {
                R g[12], xg[12], F[4], vp;
                bool xok;
                if (!gather_at(px, pth, pph, g, xg, xok)) { bad = true; break; }
                if (stage == 0 && (flags & GC_FLAG_PENDING)) collide(g);
                if (FULL && !xok) { bad = true; break; }   // after the collision, as the field's own check
                rhs_at(px, pth, pu, g, xg, F, vp);
                if (stage == 2) {
                    Fs[0] = F[0]; Fs[1] = F[1]; Fs[2] = F[2]; Fs[3] = F[3];
                    vps = EXT ? path_speed<R>(vp, g, vw) : vp;
                    break;
                }
                if (stage == 0) {
                    Fn[0] = F[0]; Fn[1] = F[1]; Fn[2] = F[2]; Fn[3] = F[3];
                    vpn = EXT ? path_speed<R>(vp, g, vw) : vp;
                    if (flags & GC_FLAG_BOOTSTRAP) {
                        // backward Euler start (Sect. 2.2)
                        px = (R)X0 - h * F[0]; pth = (R)X1 - h * F[1]; pph = (R)X2 - h * F[2]; pu = (R)X3 - h * F[3];
                        stage = 1;
                        continue;
                    }
                    tau = dtp == h ? (R)1 : h * rcp_nr(dtp);
                } else {   // stage 1: F^{n-1} of the bootstrap
                    fp0 = F[0]; fp1 = F[1]; fp2 = F[2]; fp3 = F[3];
                    tau = (R)1;
                    flags &= ~GC_FLAG_BOOTSTRAP;
                }
                predict();
                stage = 2;
            }
        } else {
            // Straight-line sites: no register copies between the stages of a
            // loop (measured faster for these forms).
            {   // X^n
                R g[12], xg[12];
                bool xok;
                if (!gather_at(px, pth, pph, g, xg, xok)) {
                    bad = true;
                } else {
                    if (flags & GC_FLAG_PENDING) collide(g);
                    if (FULL && !xok) {
                        bad = true;   // after the collision, as the field's own check
                    } else {
                        R vp;
                        rhs_at(px, pth, pu, g, xg, Fn, vp);
                        vpn = EXT ? path_speed<R>(vp, g, vw) : vp;
                    }
                }
            }
            if (!bad) {
                if (flags & GC_FLAG_BOOTSTRAP) {
                    // backward Euler start (Sect. 2.2): F^{n-1} at X^n - dt F^n
                    const R bx = (R)X0 - h * Fn[0], bth = (R)X1 - h * Fn[1], bph = (R)X2 - h * Fn[2];
                    const R bu = (R)X3 - h * Fn[3];
                    R g[12], xg[12], F[4], vp;
                    bool xok;
                    if (!gather_at(bx, bth, bph, g, xg, xok) || (FULL && !xok)) {
                        bad = true;
                    } else {
                        rhs_at(bx, bth, bu, g, xg, F, vp);
                        fp0 = F[0]; fp1 = F[1]; fp2 = F[2]; fp3 = F[3];
                        tau = (R)1;
                        flags &= ~GC_FLAG_BOOTSTRAP;
                    }
                } else {
                    tau = dtp == h ? (R)1 : h * rcp_nr(dtp);
                }
            }
            if (!bad) {   // X*
                predict();
                R g[12], xg[12], vp;
                bool xok;
                if (!gather_at(px, pth, pph, g, xg, xok) || (FULL && !xok)) {
                    bad = true;
                } else {
                    rhs_at(px, pth, pu, g, xg, Fs, vp);
                    vps = EXT ? path_speed<R>(vp, g, vw) : vp;
                }
            }
        }
        if (bad) { status = GC_NONFINITE; break; }
        // corrector, Eq. 6: dt/(6(1+tau)) [(1+tau)(3+tau) F^n + (3+2 tau) F* - tau^2 F^{n-1}]
        const R cf = tau == (R)1 ? h * (R)(1.0 / 12.0) : h * rcp_nr((R)6 * ((R)1 + tau));
        const R an = ((R)1 + tau) * ((R)3 + tau), as = (R)3 + (R)2 * tau, ap = tau * tau;
        const R e0 = cf * (an * Fn[0] + as * Fs[0] - ap * fp0);
        const R e1 = cf * (an * Fn[1] + as * Fs[1] - ap * fp1);
        const R e2 = cf * (an * Fn[2] + as * Fs[2] - ap * fp2);
        const R e3 = cf * (an * Fn[3] + as * Fs[3] - ap * fp3);
        // path along the field line over the step (trapezoid of |v_par|), Eq. 9
        if (scatter) {
            s += (R)0.5 * (fabs(vpn) + fabs(vps)) * h;
            if (s >= ell) flags |= GC_FLAG_PENDING;
        }
        A n0, n1, n2, n3;
        A nc0 = c0, nc1 = c1, nc2 = c2, nc3 = c3;   // new compensation terms (Kahan form)
        if (kKahan) {
            n0 = X0; n1 = X1; n2 = X2; n3 = X3;
            kahan_add(n0, nc0, (A)e0); kahan_add(n1, nc1, (A)e1);
            kahan_add(n2, nc2, (A)e2); kahan_add(n3, nc3, (A)e3);
        } else {
            n0 = X0 + (A)e0; n1 = X1 + (A)e1; n2 = X2 + (A)e2; n3 = X3 + (A)e3;
        }
        X0 = n0; X1 = n1; X2 = n2; X3 = n3;
        c0 = nc0; c1 = nc1; c2 = nc2; c3 = nc3;
        fp0 = Fn[0]; fp1 = Fn[1]; fp2 = Fn[2]; fp3 = Fn[3];
        dtp = h;
        if (kKahan) kahan_add(T, cT, (A)h);
        else T += (A)a.dt;
        step += 1;
        if (!(isfinite(n0) && isfinite(n1) && isfinite(n2) && isfinite(n3))) { status = GC_NONFINITE; break; }
        const double r = (double)X0, th = (double)X1;
        if (r < r_in || r > r_out || th < th_lo || th > th_hi) {
            if (!EXT || (int64_t)step >= e.rebirth_steps) { status = GC_EXITED; break; }
            // rebirth (continuous injection, Sect. 3): the next generation starts
            // from the injection state with its own generator stream
            const uint32_t gen = (flags >> GC_FLAG_GEN_SHIFT) + 1;
            const BirthState b = rebirth_state<FDT>(a.fdev, a.ens + eidx, pid, gen);
            X0 = (A)b.r; X1 = (A)b.th; X2 = (A)b.ph; X3 = (A)b.u;
            c0 = 0; c1 = 0; c2 = 0; c3 = 0; cT = 0; T = 0;
            fp0 = 0; fp1 = 0; fp2 = 0; fp3 = 0;
            mu = (R)b.mu; dtp = 0; s = 0; ell = (R)b.ell;
            k = 0;
            flags = GC_FLAG_BOOTSTRAP | (gen << GC_FLAG_GEN_SHIFT);
            birth = step;
            reborn = true;
            if (a.log_depth > 0 && gl == 0) {
                uint32_t *row = a.log + (size_t)gid * a.log_depth;
                for (int j = 0; j < a.log_depth; ++j) row[j] = 0xFFFFFFFFu;
            }
            if (b.status != GC_ACTIVE) { status = b.status; break; }
        }
        if (e.max_steps > 0 && (int64_t)step >= e.max_steps) { status = GC_FINISHED; break; }
    }
    if (gl != 0) return 0;
    st.r[slot] = (double)X0; st.th[slot] = (double)X1; st.ph[slot] = (double)X2; st.u[slot] = (double)X3;
    if (kKahan) {
        st.cr[slot] = (double)c0; st.cth[slot] = (double)c1; st.cph[slot] = (double)c2;
        st.cu[slot] = (double)c3; st.ct[slot] = (double)cT;
    }
    st.t[slot] = (double)T;
    st.fr[slot] = (double)fp0; st.fth[slot] = (double)fp1; st.fph[slot] = (double)fp2; st.fu[slot] = (double)fp3;
    st.mu[slot] = (double)mu; st.dtp[slot] = (double)dtp; st.s[slot] = (double)s; st.ell[slot] = (double)ell;
    st.k[slot] = k; st.flags[slot] = flags; st.status[slot] = status; st.step[slot] = step;
    // (in place these rewrite the values loaded: no branch, and no flag kept over the loop)
    st.id[slot] = pid; st.ens[slot] = ens_raw; st.gid[slot] = gid;
    st.birth[slot] = reborn ? birth : birth0;
    return step - step0;
}

// Grid form: one slot per G lanes.  Workgroups are dispatched round-robin over
// the 8 XCDs.  Only the first ceil(G n_active / blockDim) workgroups have work
// (active particles fill a prefix of the slots after reordering); the remap
// gives each XCD a contiguous range of that prefix, so that (with cell-sorted
// slots) its L2 holds the field cells of its own particles, and every XCD gets
// an equal share however small the active prefix is.
template <int PREC, int FDT, int MODE, int FORM, bool TAME = false>
__device__ __forceinline__ void push_grid(const PushArgs &a) {
    constexpr uint32_t G = FORM == kFormQuad ? 4 : 1;          // lanes per particle
    const uint32_t n = *a.n_active;
    const uint32_t per_block = blockDim.x / G;                // particles per workgroup
    const uint32_t nb = (n + per_block - 1) / per_block, b = blockIdx.x;
    if (b >= nb) return;
    const uint32_t q = nb >> 3, rem = nb & 7u, xcd = b & 7u, pos = b >> 3;
    const uint32_t lb = (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) + pos;
    const uint32_t slot = lb * per_block + threadIdx.x / G;
    uint32_t taken = 0;
    if (slot < n) taken = advance_slot<PREC, FDT, MODE, FORM, TAME>(a, slot, threadIdx.x % G);
    count_steps(a, taken);
}

// Throughput form: at most 256 registers per lane (two wavefronts per SIMD).
template <int PREC, int FDT, int MODE, bool TAME>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_push(PushArgs a) {
    push_grid<PREC, FDT, MODE, kFormThroughput, TAME>(a);
}

// Latency forms, for fewer active particles than fill the machine: a
// wavefront's step time is then its gathers' latency, set by the round trips
// and by how many distinct cache lines its load instructions touch.  The
// all-pairs form has each gather in one round trip; the quad form also spreads
// the particles over four times as many wavefronts (and compute units).
template <int PREC, int FDT, int MODE, bool TAME>
__global__ __launch_bounds__(256) void k_push_allpairs(PushArgs a) {
    push_grid<PREC, FDT, MODE, kFormAllPairs, TAME>(a);
}

template <int PREC, int FDT, int MODE, bool TAME>
__global__ __launch_bounds__(256) void k_push_quad(PushArgs a) {
    push_grid<PREC, FDT, MODE, kFormQuad, TAME>(a);
}

// Persistent forms: a fixed grid pulls tiles of consecutive slots from an
// atomic counter until the tiles run out (every workgroup reaches the exit).
// A tile holds a.tile particles, fewer when the live prefix would not give
// every workgroup a tile (down to one particle per thread, or per quad), so
// that a thinning population stays spread over the machine instead of
// queueing behind few workgroups.
//
// With a tail threshold T = a.tail > 0 each chunk launches the throughput,
// all-pairs and four-lanes-per-particle kernels in turn, and the live count on
// the device (written by the reorder) selects the one that works, the others
// returning at once: T and more, the throughput form; [T/kQuadShare, T), all
// pairs (for the full equations, [0, T)); below it, four lanes per particle.  These
// are the forms of the eager tail policy, chosen on the device so that a
// captured graph follows the count without a host read-back.  Steps are
// counted per form (a.steps_done + form).
template <int PREC, int FDT, int MODE, int FORM, bool TAME = false>
__device__ __forceinline__ void push_persistent(const PushArgs &a) {
    __shared__ uint32_t s_tile;
    const uint32_t n = *a.n_active;
    const uint32_t T = a.tail;
    const uint32_t q4 = MODE == 2 ? 0u : T / kQuadShare;      // the full equations have no quad form
    const uint32_t lo = FORM == kFormThroughput ? T : (FORM == kFormAllPairs ? q4 : 0u);
    const uint32_t hi = FORM == kFormThroughput ? 0xFFFFFFFFu : (FORM == kFormAllPairs ? T : q4);
    if (n < lo || n >= hi) return;
    constexpr uint32_t G = FORM == kFormQuad ? 4 : 1;          // lanes per particle
    const uint32_t per = blockDim.x / G;                       // particles per workgroup round
    const uint32_t share = ((n + gridDim.x - 1) / gridDim.x + per - 1) / per * per;
    const uint32_t tile = min(max((uint32_t)a.tile, per), max(per, share));
    const uint32_t ntiles = (n + tile - 1) / tile;
    uint32_t taken = 0;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t t = s_tile;
        __syncthreads();
        if (t >= ntiles) break;
        const uint32_t end = min(n, (t + 1) * tile);
        for (uint32_t slot = t * tile + threadIdx.x / G; slot < end; slot += per)
            taken += advance_slot<PREC, FDT, MODE, FORM, TAME>(a, slot, threadIdx.x % G);
    }
    count_steps(a.steps_done + FORM, taken);
}

template <int PREC, int FDT, int MODE, bool TAME>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_push_persistent(PushArgs a) {
    push_persistent<PREC, FDT, MODE, kFormThroughput, TAME>(a);
}

template <int PREC, int FDT, int MODE, bool TAME>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_push_persistent_allpairs(PushArgs a) {
    push_persistent<PREC, FDT, MODE, kFormAllPairs, TAME>(a);
}

template <int PREC, int FDT, int MODE, bool TAME>
__global__ __launch_bounds__(256) void k_push_persistent_quad(PushArgs a) {
    push_persistent<PREC, FDT, MODE, kFormQuad, TAME>(a);
}


template <int PREC, int FDT, int MODE, bool TAME>
static hipError_t launch_rt(const PushArgs &a, int block, bool persistent, int form, int grid_blocks, hipStream_t s,
                           LaunchEvents ev) {
    if (persistent) {
        const bool quad = a.tail > 0 && MODE != 2;
        launch_timed((k_push_persistent<PREC, FDT, MODE, TAME>), dim3(grid_blocks), dim3(block), s, ev.start,
                     a.tail > 0 ? nullptr : ev.stop, a);
        if (a.tail > 0) {
            launch_timed((k_push_persistent_allpairs<PREC, FDT, MODE, TAME>), dim3(grid_blocks), dim3(block), s, nullptr,
                         quad ? nullptr : ev.stop, a);
            if (quad) {  // 256-thread workgroups (64 particles per round), as the grid quad form
                launch_timed((k_push_persistent_quad<PREC, FDT, MODE == 2 ? 1 : MODE, TAME>),
                             dim3((uint32_t)grid_blocks * block / 256), dim3(256), s, nullptr, ev.stop, a);
            }
        }
    } else {
        const uint32_t nb = (a.n_slots + block - 1) / block;
        if (nb == 0) {
            if (ev.start) (void)hipEventRecord(ev.start, s);
            if (ev.stop) (void)hipEventRecord(ev.stop, s);
            return hipGetLastError();
        }
        if (form == kFormQuad && MODE != 2) {
            // 256-thread workgroups whatever the block size (64 particles each;
            // measured faster for this form than 64 threads)
            const uint32_t qb = (4 * a.n_slots + 255) / 256;
            launch_timed((k_push_quad<PREC, FDT, MODE == 2 ? 1 : MODE, TAME>), dim3(qb), dim3(256), s, ev.start,
                         ev.stop, a);
        } else if (form != kFormThroughput)
            launch_timed((k_push_allpairs<PREC, FDT, MODE, TAME>), dim3(nb), dim3(block), s, ev.start, ev.stop, a);
        else
            launch_timed((k_push<PREC, FDT, MODE, TAME>), dim3(nb), dim3(block), s, ev.start, ev.stop, a);
    }
    return hipGetLastError();
}

// The tame instantiations (FieldDev::tame) for the reduced equations; the
// full equations test every gather (their extra node array is not scanned).
template <int PREC, int FDT, int MODE>
static hipError_t launch_r(const PushArgs &a, int block, bool persistent, int form, int grid_blocks, hipStream_t s,
                           LaunchEvents ev) {
    if constexpr (MODE != 2)
        if (a.f.tame) return launch_rt<PREC, FDT, MODE, true>(a, block, persistent, form, grid_blocks, s, ev);
    return launch_rt<PREC, FDT, MODE, false>(a, block, persistent, form, grid_blocks, s, ev);
}

template <int PREC, int FDT>
static hipError_t launch_t(const PushArgs &a, int block, bool persistent, int form, int grid_blocks, hipStream_t s,
                           LaunchEvents ev) {
    switch (a.mode) {
        case 0: return launch_r<PREC, FDT, 0>(a, block, persistent, form, grid_blocks, s, ev);
        case 1: return launch_r<PREC, FDT, 1>(a, block, persistent, form, grid_blocks, s, ev);
        default: return launch_r<PREC, FDT, 2>(a, block, persistent, form, grid_blocks, s, ev);
    }
}

template <int PREC>
static hipError_t launch_p(const PushArgs &a, int block, bool persistent, int form, int grid_blocks, hipStream_t s,
                           LaunchEvents ev) {
    switch (a.f.dtype) {
        case GC_F64: return launch_t<PREC, GC_F64>(a, block, persistent, form, grid_blocks, s, ev);
        case GC_F32: return launch_t<PREC, GC_F32>(a, block, persistent, form, grid_blocks, s, ev);
        case GC_F16: return launch_t<PREC, GC_F16>(a, block, persistent, form, grid_blocks, s, ev);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_push(const PushArgs &a, int precision, int block, bool persistent, int form, int grid_blocks,
                       hipStream_t s, LaunchEvents ev) {
    switch (precision) {
        case GC_PREC_F64: return launch_p<GC_PREC_F64>(a, block, persistent, form, grid_blocks, s, ev);
        case GC_PREC_F32_ACC64: return launch_p<GC_PREC_F32_ACC64>(a, block, persistent, form, grid_blocks, s, ev);
        case GC_PREC_F32_KAHAN: return launch_p<GC_PREC_F32_KAHAN>(a, block, persistent, form, grid_blocks, s, ev);
    }
    return hipErrorInvalidValue;
}

}  // namespace gc
