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

// Generator block of collision k1 (counter (id, k1, 0, 0), key (seed, ensemble)):
// new pitch cosine from a1 (Eq. 10, or Eq. 12 with the sign from a2) and the
// next free path -lambda ln(1 - a0).  Kept out of line: it runs for a few
// steps in a thousand, and inlined it would raise the push's register count.
struct CollisionDraw { double mun, ell; };

__device__ __noinline__ CollisionDraw draw_collision(uint32_t pid, uint32_t k1, uint64_t seed, uint32_t ens,
                                                     int law, double lambda) {
    const U64x4 rb = philox4x64_10(pid, k1, kPurposePath, 0, seed, ens);
    const double a0 = u01(rb.v[0]), a1 = u01(rb.v[1]), a2 = u01(rb.v[2]);
    CollisionDraw d;
    d.mun = law == 1 ? (a2 < 0.5 ? -1.0 : 1.0) * sqrt(a1) : 1.0 - 2.0 * a1;
    d.ell = -lambda * log(1.0 - a0);
    return d;
}

__device__ __forceinline__ void count_steps(const PushArgs &a, uint32_t taken) {
    // one atomic per wavefront
    uint32_t v = taken;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(a.steps_done, (unsigned long long)v);
}

}  // namespace gc
