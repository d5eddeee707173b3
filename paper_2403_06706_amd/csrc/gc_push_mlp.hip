// gc_push_mlp.hip -- the push with the neural field as field source.
#include <hip/hip_runtime.h>

#include "gc_device.h"
#include "gc_launch.h"
#include "gc_mlp.h"
#include "gc_mlp_launch.h"
#include "gc_step.h"

namespace gc {

// ---------------------------------------------------------------------------
// Push with the neural field as field source.  The same step as advance_slot,
// but the field evaluation is a workgroup-wide matrix-core product
// (mlp_block), so every thread of the workgroup takes part in every
// evaluation and the step and stage loops run in lockstep over the workgroup:
// threads without work (exited, finished their stages, or past the active
// prefix) evaluate at their last position and ignore the result.
// ---------------------------------------------------------------------------
constexpr int kPushMlpThreads = 512;   // 8 wavefronts (2 per SIMD) share the staged weights

template <int PREC>
__global__ __launch_bounds__(kPushMlpThreads) __attribute__((amdgpu_waves_per_eu(2)))
void k_push_mlp(PushArgs a, MlpArgs m) {
    using R = typename PrecT<PREC>::R;
    using A = typename PrecT<PREC>::A;
    constexpr bool kKahan = PrecT<PREC>::kKahan;
    __shared__ MlpLds<kPushMlpThreads> L;
    const uint32_t n = *a.n_active;
    const uint32_t nb = (n + blockDim.x - 1) / blockDim.x, bidx = blockIdx.x;
    if (bidx >= nb) return;                                   // whole workgroup idle
    mlp_lds_init(m, L);
    const uint32_t q8 = nb >> 3, rem = nb & 7u, xcd = bidx & 7u, pos = bidx >> 3;
    const uint32_t lb = (xcd < rem ? xcd * (q8 + 1) : rem * (q8 + 1) + (xcd - rem) * q8) + pos;
    const uint32_t slot = lb * blockDim.x + threadIdx.x;
    const SoA &st = a.st;
    const bool in_range = slot < n;
    const uint32_t ls = in_range ? slot : n - 1;              // lanes past the prefix read a valid slot
    uint32_t status = st.status[ls];
    bool alive = in_range && status == GC_ACTIVE;
    uint32_t flags = st.flags[ls], k = st.k[ls], step = st.step[ls];
    const uint32_t step0 = step;
    const EnsDev e = a.ens[min(st.ens[ls], (uint32_t)(kMaxEnsembles - 1))];
    const uint32_t pid = st.id[ls];
    A X0 = (A)st.r[ls], X1 = (A)st.th[ls], X2 = (A)st.ph[ls], X3 = (A)st.u[ls];
    A T = (A)st.t[ls];
    A c0 = 0, c1 = 0, c2 = 0, c3 = 0, cT = 0;
    if (kKahan) {
        c0 = (A)st.cr[ls]; c1 = (A)st.cth[ls]; c2 = (A)st.cph[ls]; c3 = (A)st.cu[ls]; cT = (A)st.ct[ls];
    }
    R fp0 = (R)st.fr[ls], fp1 = (R)st.fth[ls], fp2 = (R)st.fph[ls], fp3 = (R)st.fu[ls];
    R mu = (R)st.mu[ls], dtp = (R)st.dtp[ls], s = (R)st.s[ls], ell = (R)st.ell[ls];
    const R qm = (R)e.qm, iqm = (R)e.iqm;
    const bool drift_free = e.drift_free != 0;
    const bool scatter = e.lambda > 0.0;
    const R h = (R)a.dt;
    const double r_in = e.r_in, r_out = e.r_out, th_lo = a.f.th_lo, th_hi = a.f.th_hi;

    // Per-lane stage machine: each lane walks through its own stages (X^n, the
    // bootstrap X^{n-1}, X*) and steps; every iteration evaluates the network
    // once for the whole workgroup, at each lane's current point, until every
    // lane has taken its steps.  A lane's bootstrap therefore costs the
    // workgroup one evaluation only when that lane is the last to finish.
    int remaining = alive ? a.n_steps : 0;
    bool active = remaining > 0;
    R Fn[4] = {0, 0, 0, 0}, vpn = 0, tau = 1;
    R mun = 0, ell_new = 0;
    if (active && (flags & GC_FLAG_PENDING)) {
        const CollisionDraw d = draw_collision(pid, k + 1, flags >> GC_FLAG_GEN_SHIFT, e.seed, e.ensemble,
                                               e.scatter_law, e.lambda);
        mun = (R)d.mun;
        ell_new = (R)d.ell;
    }
    R px = (R)X0, pth = (R)X1, pph = (R)X2, pu = (R)X3;
    int stage = 0;
    while (__syncthreads_or(active)) {                        // uniform over the workgroup
        float y[kMlpOut], dy[3][kMlpOut];
        mlp_block<kPushMlpThreads, kMlpDepth + 1>(m, (float)px, (float)pth, (float)pph, L, y, dy);
        if (!active) continue;
        R g[12];
        if (!mlp_assemble<R>(m, px, pth, y, dy, g)) { status = GC_NONFINITE; active = false; continue; }
        if (stage == 0 && (flags & GC_FLAG_PENDING)) {
            const R B = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            const R p2 = pu * pu + (R)2 * mu * B;
            X3 = (A)(mun * sqrt(p2));
            c3 = 0;
            pu = (R)X3;
            mu = p2 * ((R)1 - mun * mun) / ((R)2 * B);
            ell = ell_new;
            s = 0;
            k += 1;
            flags = (flags | GC_FLAG_BOOTSTRAP) & ~GC_FLAG_PENDING;
            if (a.log_depth > 0 && k <= (uint32_t)a.log_depth)
                a.log[(size_t)st.gid[ls] * a.log_depth + (k - 1)] = step;
        }
        R F[4], vp;
        gc_rhs<R>(px, pth, pu, mu, qm, iqm, drift_free, g, F, vp);
        if (stage == 2) {
            // corrector (F is F*), path, exit and stop tests; then the next step
            const R cf = tau == (R)1 ? h * (R)(1.0 / 12.0) : h * rcp_nr((R)6 * ((R)1 + tau));
            const R an = ((R)1 + tau) * ((R)3 + tau), as = (R)3 + (R)2 * tau, ap = tau * tau;
            const R e0 = cf * (an * Fn[0] + as * F[0] - ap * fp0);
            const R e1 = cf * (an * Fn[1] + as * F[1] - ap * fp1);
            const R e2 = cf * (an * Fn[2] + as * F[2] - ap * fp2);
            const R e3 = cf * (an * Fn[3] + as * F[3] - ap * fp3);
            if (scatter) {
                s += (R)0.5 * (fabs(vpn) + fabs(vp)) * h;
                if (s >= ell) flags |= GC_FLAG_PENDING;
            }
            if (kKahan) {
                kahan_add(X0, c0, (A)e0); kahan_add(X1, c1, (A)e1); kahan_add(X2, c2, (A)e2); kahan_add(X3, c3, (A)e3);
                kahan_add(T, cT, (A)h);
            } else {
                X0 += (A)e0; X1 += (A)e1; X2 += (A)e2; X3 += (A)e3;
                T += (A)a.dt;
            }
            fp0 = Fn[0]; fp1 = Fn[1]; fp2 = Fn[2]; fp3 = Fn[3];
            dtp = h;
            step += 1;
            if (!(isfinite(X0) && isfinite(X1) && isfinite(X2) && isfinite(X3))) { status = GC_NONFINITE; active = false; continue; }
            const double r = (double)X0, th = (double)X1;
            if (r < r_in || r > r_out || th < th_lo || th > th_hi) { status = GC_EXITED; active = false; continue; }
            if (e.max_steps > 0 && (int64_t)step >= e.max_steps) { status = GC_FINISHED; active = false; continue; }
            if (--remaining == 0) { active = false; continue; }
            stage = 0;
            tau = 1;
            mun = 0;
            ell_new = 0;
            if (flags & GC_FLAG_PENDING) {
                const CollisionDraw d = draw_collision(pid, k + 1, flags >> GC_FLAG_GEN_SHIFT, e.seed, e.ensemble,
                                               e.scatter_law, e.lambda);
                mun = (R)d.mun;
                ell_new = (R)d.ell;
            }
            px = (R)X0; pth = (R)X1; pph = (R)X2; pu = (R)X3;
            continue;
        }
        if (stage == 0) {
            Fn[0] = F[0]; Fn[1] = F[1]; Fn[2] = F[2]; Fn[3] = F[3];
            vpn = vp;
            if (flags & GC_FLAG_BOOTSTRAP) {
                px = (R)X0 - h * F[0]; pth = (R)X1 - h * F[1]; pph = (R)X2 - h * F[2]; pu = (R)X3 - h * F[3];
                stage = 1;
                continue;
            }
            tau = dtp == h ? (R)1 : h * rcp_nr(dtp);
        } else {
            fp0 = F[0]; fp1 = F[1]; fp2 = F[2]; fp3 = F[3];
            tau = (R)1;
            flags &= ~GC_FLAG_BOOTSTRAP;
        }
        // predictor (Eq. 5)
        const R wn = (R)1 + (R)0.5 * tau, wq = (R)0.5 * tau;
        const R d0 = h * (wn * Fn[0] - wq * fp0), d1 = h * (wn * Fn[1] - wq * fp1);
        const R d2 = h * (wn * Fn[2] - wq * fp2), d3 = h * (wn * Fn[3] - wq * fp3);
        if (kKahan) {
            px = (R)(X0 + (d0 - c0)); pth = (R)(X1 + (d1 - c1)); pph = (R)(X2 + (d2 - c2)); pu = (R)(X3 + (d3 - c3));
        } else {
            px = (R)(X0 + (A)d0); pth = (R)(X1 + (A)d1); pph = (R)(X2 + (A)d2); pu = (R)(X3 + (A)d3);
        }
        stage = 2;
    }
    uint32_t taken = 0;
    if (in_range && step != step0 || (in_range && status != st.status[ls])) {
        st.r[slot] = (double)X0; st.th[slot] = (double)X1; st.ph[slot] = (double)X2; st.u[slot] = (double)X3;
        if (kKahan) {
            st.cr[slot] = (double)c0; st.cth[slot] = (double)c1; st.cph[slot] = (double)c2;
            st.cu[slot] = (double)c3; st.ct[slot] = (double)cT;
        }
        st.t[slot] = (double)T;
        st.fr[slot] = (double)fp0; st.fth[slot] = (double)fp1; st.fph[slot] = (double)fp2; st.fu[slot] = (double)fp3;
        st.mu[slot] = (double)mu; st.dtp[slot] = (double)dtp; st.s[slot] = (double)s; st.ell[slot] = (double)ell;
        st.k[slot] = k; st.flags[slot] = flags; st.status[slot] = status; st.step[slot] = step;
        taken = step - step0;
    }
    count_steps(a, taken);
}

template <int PREC>
static hipError_t launch_mlp_t(const PushArgs &a, const MlpArgs &m, hipStream_t s) {
    const uint32_t nb = (a.n_slots + kPushMlpThreads - 1) / kPushMlpThreads;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_push_mlp<PREC>), dim3(nb), dim3(kPushMlpThreads), 0, s, a, m);
    return hipGetLastError();
}

hipError_t launch_push_mlp(const PushArgs &a, const MlpArgs &m, int precision, hipStream_t s) {
    switch (precision) {
        case GC_PREC_F64: return launch_mlp_t<GC_PREC_F64>(a, m, s);
        case GC_PREC_F32_ACC64: return launch_mlp_t<GC_PREC_F32_ACC64>(a, m, s);
        case GC_PREC_F32_KAHAN: return launch_mlp_t<GC_PREC_F32_KAHAN>(a, m, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gc
