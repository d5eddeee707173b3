// gc_probe.hip -- gather ceiling: the field gathers of the push without its
// arithmetic, for the roofline denominator of the grid push.
//
// Each active particle moves on the straight line X + k dt F^{n-1} (its last
// right-hand side: along its field line, at its speed) and makes the push's two
// gathers per step, at X^n and half a step ahead.  Same packed layout, same
// cell-sorted slot order, same XCD-aware workgroup remap and the same gather
// code as the push; no right-hand side, no integrator, no state written.
#include <hip/hip_runtime.h>

#include "gc_device.h"
#include "gc_launch.h"
#include "gc_step.h"

namespace gc {

template <int FDT, bool TAME>
__global__ __launch_bounds__(256) void k_gather_probe(PushArgs a, double *sink) {
    const uint32_t n = *a.n_active;
    const uint32_t nb = (n + blockDim.x - 1) / blockDim.x, b = blockIdx.x;
    if (b >= nb) return;
    const uint32_t q = nb >> 3, rem = nb & 7u, xcd = b & 7u, pos = b >> 3;
    const uint32_t lb = (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) + pos;
    const uint32_t slot = lb * blockDim.x + threadIdx.x;
    count_steps(a, slot < n ? (uint32_t)a.n_steps : 0u);   // particle-steps of the probe
    if (slot >= n) return;
    const SoA &st = a.st;
    double x = st.r[slot], y = st.th[slot], z = st.ph[slot];
    const double h = a.dt;
    double vx = st.fr[slot], vy = st.fth[slot], vz = st.fph[slot];
    if (!(isfinite(vx) && isfinite(vy) && isfinite(vz))) vx = vy = vz = 0.0;
    double acc = 0.0;
    for (int it = 0; it < a.n_steps; ++it) {
        double g[12];
        if (gather<FDT, double, false, TAME>(a.f, x, y, z, g)) acc += g[0] + g[5] + g[11];
        if (gather<FDT, double, false, TAME>(a.f, x + 0.5 * h * vx, y + 0.5 * h * vy, z + 0.5 * h * vz, g))
            acc += g[1] + g[6] + g[9];
        x += h * vx;
        y += h * vy;
        z += h * vz;
    }
    sink[slot] = acc;
}

hipError_t launch_gather_probe(const PushArgs &a, double *sink, int block, hipStream_t s) {
    const uint32_t nb = (a.n_slots + block - 1) / block;      // the push's workgroup size
    if (nb == 0) return hipSuccess;
    // the push's gathers: without the finiteness test on a tame field
    const bool t = a.f.tame != 0;
    switch (a.f.dtype) {
        case GC_F64:
            if (t) hipLaunchKernelGGL((k_gather_probe<GC_F64, true>), dim3(nb), dim3(block), 0, s, a, sink);
            else hipLaunchKernelGGL((k_gather_probe<GC_F64, false>), dim3(nb), dim3(block), 0, s, a, sink);
            break;
        case GC_F32:
            if (t) hipLaunchKernelGGL((k_gather_probe<GC_F32, true>), dim3(nb), dim3(block), 0, s, a, sink);
            else hipLaunchKernelGGL((k_gather_probe<GC_F32, false>), dim3(nb), dim3(block), 0, s, a, sink);
            break;
        default:
            if (t) hipLaunchKernelGGL((k_gather_probe<GC_F16, true>), dim3(nb), dim3(block), 0, s, a, sink);
            else hipLaunchKernelGGL((k_gather_probe<GC_F16, false>), dim3(nb), dim3(block), 0, s, a, sink);
            break;
    }
    return hipGetLastError();
}

}  // namespace gc
