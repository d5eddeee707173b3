// gc_kernels.hip -- injection, field packing, state copies, fills.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gc_device.h"
#include "gc_launch.h"
#include "gc_step.h"

namespace gc {

// ---------------------------------------------------------------------------
// Field packing: [nr][nth][nph][12] float64 (staged on the device) -> the
// blocked layout of field_layout in the storage type (records == 0), or node
// records [nr][nth][nph+1][12] (records != 0); the extra phi node k = nph
// repeats node 0, padding nodes are zero.  FP16 stores v / scale rounded once
// from double to half.
// ---------------------------------------------------------------------------
__global__ void k_pack_field(const double *src, void *dst, int nr, int nth, int nph, int dtype, int records,
                             const float *inv_scale_in) {
    const FieldLayout L = field_layout(nr, nth, nph, dtype);
    const uint64_t nI = L.cs / (kLayB * L.W), nK = L.js / L.ks;
    const uint64_t total = records ? (uint64_t)nr * nth * (nph + 1) * 12 : L.total;
    for (uint64_t o = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; o < total;
         o += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t i, j, k;
        int comp;
        if (records) {
            comp = (int)(o % 12);
            const uint64_t node = o / 12;
            k = node % (nph + 1);
            j = (node / (nph + 1)) % nth;
            i = node / ((uint64_t)(nph + 1) * nth);
        } else {
            uint64_t t = o / L.W;
            const uint64_t e = o % L.W;
            const uint64_t ii = t % kLayBr;
            t /= kLayBr;
            const uint64_t kk = t % kLayBk;
            t /= kLayBk;
            const uint64_t I = t % nI;
            t /= nI;
            const uint64_t c = t % L.nch;
            t /= L.nch;
            const uint64_t K = t % nK;
            j = t / nK;
            i = I * kLayBr + ii;
            k = K * kLayBk + kk;
            comp = (int)(c * L.W + e);
        }
        double v = 0.0;
        if (i < (uint64_t)nr && k <= (uint64_t)nph)
            v = src[((i * nth + j) * nph + (k == (uint64_t)nph ? 0 : k)) * 12 + comp];
        if (dtype == GC_F64) static_cast<double *>(dst)[o] = v;
        else if (dtype == GC_F32) static_cast<float *>(dst)[o] = (float)v;
        else   // one rounding, double -> half (to nearest even)
            static_cast<__half *>(dst)[o] = __half_raw{static_cast<_Float16>(v * (double)inv_scale_in[comp])};
    }
}

hipError_t launch_pack_field(const double *src, void *dst, int nr, int nth, int nph, int dtype, int records,
                             const float *inv_scale, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_field, dim3(2048), dim3(256), 0, s, src, dst, nr, nth, nph, dtype, records, inv_scale);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Injection (Sect. 3): one particle per lane, FP64.
// ---------------------------------------------------------------------------
template <int FDT>
__global__ void k_inject(SoA st, FieldDev f, EnsDev e, uint32_t n0, uint32_t n, uint32_t first_id, uint32_t eidx) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t slot = n0 + i, pid = first_id + i;
    const BirthState b = birth_state<FDT>(f, e, pid, 0);
    st.r[slot] = b.r; st.th[slot] = b.th; st.ph[slot] = b.ph; st.u[slot] = b.u; st.mu[slot] = b.mu;
    st.fr[slot] = 0.0; st.fth[slot] = 0.0; st.fph[slot] = 0.0; st.fu[slot] = 0.0;
    st.dtp[slot] = 0.0; st.s[slot] = 0.0; st.ell[slot] = b.ell; st.t[slot] = 0.0;
    st.cr[slot] = 0.0; st.cth[slot] = 0.0; st.cph[slot] = 0.0; st.cu[slot] = 0.0; st.ct[slot] = 0.0;
    st.k[slot] = 0; st.flags[slot] = GC_FLAG_BOOTSTRAP; st.status[slot] = b.status; st.step[slot] = 0;
    st.id[slot] = pid; st.ens[slot] = eidx; st.gid[slot] = slot; st.birth[slot] = 0;
}

hipError_t launch_inject(const SoA &st, const FieldDev &f, const EnsDev &e, uint32_t n0, uint32_t n,
                         uint32_t first_id, uint32_t eidx, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const dim3 grid((n + 255) / 256), block(256);
    switch (f.dtype) {
        case GC_F64: hipLaunchKernelGGL(k_inject<GC_F64>, grid, block, 0, s, st, f, e, n0, n, first_id, eidx); break;
        case GC_F32: hipLaunchKernelGGL(k_inject<GC_F32>, grid, block, 0, s, st, f, e, n0, n, first_id, eidx); break;
        default:     hipLaunchKernelGGL(k_inject<GC_F16>, grid, block, 0, s, st, f, e, n0, n, first_id, eidx); break;
    }
    return hipGetLastError();
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

static unsigned grid_for(size_t n, unsigned block) {
    size_t g = (n + block - 1) / block;
    if (g > 4096) g = 4096;
    return g == 0 ? 1u : (unsigned)g;
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// State export / import in global injection order.
// ---------------------------------------------------------------------------
#define GC_FOR_DOUBLES(X) X(r) X(th) X(ph) X(u) X(mu) X(fr) X(fth) X(fph) X(fu) X(dtp) X(s) X(ell) X(t) \
                          X(cr) X(cth) X(cph) X(cu) X(ct)
#define GC_FOR_U32(X) X(k) X(flags) X(status) X(step) X(id) X(ens) X(birth)

__global__ void k_state_out(SoA st, gc_state_view dst, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t g = st.gid[i];
#define OUT_(name) if (dst.name) dst.name[g] = st.name[i];
    GC_FOR_DOUBLES(OUT_)
    GC_FOR_U32(OUT_)
#undef OUT_
}

__global__ void k_state_in(SoA st, gc_state_view src, uint32_t n) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
#define IN_(name) st.name[g] = src.name[g];
    GC_FOR_DOUBLES(IN_)
    GC_FOR_U32(IN_)
#undef IN_
    st.gid[g] = g;
}

hipError_t launch_state_out(const SoA &st, const gc_state_view &dst, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_state_out, dim3((n + 255) / 256), dim3(256), 0, s, st, dst, n);
    return hipGetLastError();
}
hipError_t launch_state_in(const SoA &st, const gc_state_view &src, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_state_in, dim3((n + 255) / 256), dim3(256), 0, s, st, src, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain streaming copy for counter calibration and the achievable HBM rate:
// each thread keeps four independent 16-byte loads in flight per iteration.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_copy_probe(uint4 *dst, const uint4 *src, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

hipError_t launch_copy_probe(void *dst, const void *src, size_t n_bytes, hipStream_t s) {
    const size_t n16 = n_bytes / 16;
    if (n16 == 0) return hipSuccess;
    const size_t want = (n16 + 4 * 256 - 1) / (4 * 256);           // four pieces per thread
    const unsigned grid = (unsigned)std::min<size_t>(std::max<size_t>(want, 1), 32768);
    hipLaunchKernelGGL(k_copy_probe, dim3(grid), dim3(256), 0, s, static_cast<uint4 *>(dst),
                       static_cast<const uint4 *>(src), n16);
    return hipGetLastError();
}

}  // namespace gc
