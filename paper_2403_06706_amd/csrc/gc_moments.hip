// gc_moments.hip -- snapshot statistics of the particle state (Sect. 3:
// <sin^2 alpha>(r), energy versus age near 1 AU, pitch-cosine distributions,
// and counts by status).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gc_device.h"
#include "gc_launch.h"

namespace gc {

// ---------------------------------------------------------------------------
// Moments: per-block 64-bit histograms in LDS, merged with global atomics.
// Every contribution is an integer, so the result does not depend on order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long fixp(double x, double scale) {
    return (unsigned long long)(long long)floor(x * scale);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <int FDT>
__global__ void k_moments(SoA st, FieldDev f, const EnsDev *ens, uint32_t n_all, MomDev m, unsigned long long *out,
                          const uint32_t *n_scan, const unsigned long long *dead) {
    extern __shared__ unsigned long long h[];
    const uint32_t n = n_scan ? *n_scan : n_all;
    if (blockIdx.x > 0 && blockIdx.x * blockDim.x >= n) return;   // nothing to read (uniform)
    for (int i = threadIdx.x; i < m.total; i += blockDim.x) h[i] = 0ull;
    __syncthreads();
    unsigned long long *rb = h + 8;
    unsigned long long *mh = rb + 3 * m.n_rbins;
    unsigned long long *eh = mh + m.n_mubins;
    // the eight scalar moments are summed in registers, then once per wavefront
    unsigned long long acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t status = st.status[i];
        if (status <= GC_NONFINITE) acc[status] += 1;
        acc[4] += st.k[i];
        acc[5] += st.step[i];
        if (status != GC_ACTIVE) continue;
        const double r = st.r[i], th = st.th[i], ph = st.ph[i], u = st.u[i], mu = st.mu[i], t = st.t[i];
        const uint32_t k = st.k[i];
        acc[6] += fixp(r / m.len_unit, 4294967296.0);
        if (k >= 1) acc[7] += 1;
        if (st.birth[i] < m.min_birth) continue;
        double g[12];
        if (!gather<FDT, double>(f, r, th, ph, g)) continue;
        const double B = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        const double p2 = u * u + 2.0 * mu * B;                // (|p|/m)^2
        const double pm = sqrt(p2);
        const double cosa = pm > 0.0 ? u / pm : 1.0;
        const double sin2 = 1.0 - cosa * cosa;
        const double gamma = sqrt(1.0 + p2 * kInvC2);
        const double ekin = (gamma - 1.0) * ens[min(st.ens[i], (uint32_t)(kMaxEnsembles - 1))].m * kC * kC / m.e_unit;
        if (m.n_rbins > 0) {
            const double x = (r - m.r_lo) / (m.r_hi - m.r_lo) * m.n_rbins;
            if (x >= 0.0 && x < (double)m.n_rbins) {
                const int bi = (int)floor(x);
                atomicAdd(&rb[3 * bi + 0], 1ull);
                atomicAdd(&rb[3 * bi + 1], fixp(sin2, 4294967296.0));
                atomicAdd(&rb[3 * bi + 2], fixp(ekin, 65536.0));
            }
        }
        if (r < m.sel_r_lo || r >= m.sel_r_hi) continue;
        if (m.n_mubins > 0 && t >= m.age_lo && t < m.age_hi && (int64_t)k >= (int64_t)m.min_collisions) {
            const double x = (cosa + 1.0) * 0.5 * m.n_mubins;
            int bi = (int)floor(x);
            bi = bi < 0 ? 0 : (bi >= m.n_mubins ? m.n_mubins - 1 : bi);
            atomicAdd(&mh[bi], 1ull);
        }
        if (m.n_agebins > 0 && m.n_ebins > 0) {
            const double xa = t / m.age_max * m.n_agebins;
            const double xe = (ekin - m.e_lo) / (m.e_hi - m.e_lo) * m.n_ebins;
            if (xa >= 0.0 && xa < (double)m.n_agebins && xe >= 0.0 && xe < (double)m.n_ebins)
                atomicAdd(&eh[(int)floor(xa) * m.n_ebins + (int)floor(xe)], 1ull);
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const unsigned long long v = wave_sum(acc[q]);
        if ((threadIdx.x & 63u) == 0 && v) atomicAdd(&h[q], v);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m.total; i += blockDim.x)
        if (h[i]) atomicAdd(&out[i], h[i]);
    // slots past the live prefix: their sums, kept by the reorders
    if (dead && blockIdx.x == 0 && threadIdx.x < 6 && dead[threadIdx.x]) atomicAdd(&out[threadIdx.x], dead[threadIdx.x]);
}

hipError_t launch_moments(const SoA &st, const FieldDev &f, const EnsDev *ens, uint32_t n, const MomDev &m,
                          unsigned long long *out, const uint32_t *n_scan, const unsigned long long *dead,
                          hipStream_t s) {
    hipError_t e = m.accumulate ? hipSuccess : launch_fill_u64(out, 0ull, (size_t)m.total, s);
    if (e != hipSuccess || n == 0) return e;
    const dim3 grid(std::min<uint32_t>((n + 255) / 256, 1024u)), block(256);
    const size_t lds = (size_t)m.total * sizeof(unsigned long long);
    switch (f.dtype) {
        case GC_F64: hipLaunchKernelGGL(k_moments<GC_F64>, grid, block, lds, s, st, f, ens, n, m, out, n_scan, dead); break;
        case GC_F32: hipLaunchKernelGGL(k_moments<GC_F32>, grid, block, lds, s, st, f, ens, n, m, out, n_scan, dead); break;
        default:     hipLaunchKernelGGL(k_moments<GC_F16>, grid, block, lds, s, st, f, ens, n, m, out, n_scan, dead); break;
    }
    return hipGetLastError();
}

}  // namespace gc
