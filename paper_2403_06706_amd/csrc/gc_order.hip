// gc_order.hip -- particle reordering between chunks of steps.
//
//  * cell binning: key = field cell of the particle (optionally coarsened),
//    inactive particles get the largest key; LSD radix sort (8-bit digits) of
//    (key, slot) pairs; permute the state.  Particles of one cell then sit in
//    consecutive lanes, so their trilinear gathers hit the same cache lines.
//  * compaction: stable partition active-first from wavefront ballots.
// Both produce perm[dst] = src and leave the active count on the device.
#include <hip/hip_runtime.h>

#include "gc_device.h"
#include "gc_launch.h"

namespace gc {

constexpr int kRsThreads = 256;
constexpr int kRsItems = kSortTile / kRsThreads;   // items per thread per block
constexpr int kWaves = kRsThreads / 64;

__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t lane = threadIdx.x & 63u;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cell_keys(SoA st, FieldDev f, const uint32_t *np, int coarsen,
                                                   uint32_t dead_key, uint32_t *keys, uint32_t *block_alive) {
    __shared__ uint32_t wsum[4];
    const uint32_t n = *np;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool alive = false;
    if (i < n) {
        uint32_t key = dead_key;
        if (st.status[i] == GC_ACTIVE) {
            alive = true;
            const double x = (st.r[i] - f.r_min) * f.inv_dr;
            const double y = st.th[i] * f.inv_dth - 0.5;
            const double z = st.ph[i] * f.inv_dph;
            double fi = clampr(floor(x), 0.0, (double)(f.nr - 2));
            double fj = clampr(floor(y), 0.0, (double)(f.nth - 2));
            double zf = floor(z);
            double km = zf - (double)f.nph * floor(zf * f.inv_nph);
            km = km < 0.0 ? km + f.nph : km;
            km = km >= f.nph ? km - f.nph : km;
            km = clampr(km, 0.0, (double)(f.nph - 1));
            if (!(isfinite(x) && isfinite(y) && isfinite(z))) { fi = 0.0; fj = 0.0; km = 0.0; }
            const uint32_t nthc = ((uint32_t)f.nth + (1u << coarsen) - 1) >> coarsen;
            const uint32_t nphc = ((uint32_t)f.nph + (1u << coarsen) - 1) >> coarsen;
            key = (((uint32_t)fi >> coarsen) * nthc + ((uint32_t)fj >> coarsen)) * nphc + ((uint32_t)km >> coarsen);
        }
        keys[i] = key;
    }
    const uint64_t b = __ballot(alive);
    if ((threadIdx.x & 63u) == 0) wsum[threadIdx.x >> 6] = (uint32_t)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) block_alive[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t *v, uint32_t nb, uint32_t *n_active);

hipError_t launch_cell_keys(const SoA &st, const FieldDev &f, const uint32_t *np, uint32_t n_max, int coarsen,
                            uint32_t dead_key, uint32_t *keys, uint32_t *block_alive, uint32_t *n_active,
                            hipStream_t s) {
    if (n_max == 0) return launch_fill_u32(n_active, 0u, 1, s);
    const uint32_t nb = (n_max + 255) / 256;
    hipLaunchKernelGGL(k_cell_keys, dim3(nb), dim3(256), 0, s, st, f, np, coarsen, dead_key, keys, block_alive);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, block_alive, nb, n_active);   // total -> n_active
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// LSD radix sort, one 8-bit digit per pass: histogram per block, scan per
// digit across blocks, stable scatter with per-wavefront ranking by ballots.
// counts layout: [digit][block].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint32_t *keys, const uint32_t *np, int shift,
                                                       uint32_t *counts, uint32_t nblocks) {
    __shared__ uint32_t h[256];
    const uint32_t n = *np;
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * kSortTile;
    for (int it = 0; it < kRsItems; ++it) {
        const uint32_t i = base + it * kRsThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// one workgroup per digit: exclusive scan of counts[d][0..nblocks) in place
__global__ __launch_bounds__(kRsThreads) void k_rs_scan_digit(uint32_t *counts, uint32_t nblocks, uint32_t *totals) {
    __shared__ uint32_t sh[kRsThreads];
    uint32_t *row = counts + (size_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nblocks; base += kRsThreads) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < nblocks ? row[i] : 0u;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kRsThreads; off <<= 1) {
            const uint32_t t = threadIdx.x >= (uint32_t)off ? sh[threadIdx.x - off] : 0u;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nblocks) row[i] = carry + sh[threadIdx.x] - v;
        carry += sh[kRsThreads - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint32_t *keys_in, const uint32_t *vals_in,
                                                          uint32_t *keys_out, uint32_t *vals_out,
                                                          const uint32_t *np, int shift, const uint32_t *counts,
                                                          const uint32_t *totals, uint32_t nblocks) {
    const uint32_t n = *np;
    if (blockIdx.x * kSortTile >= n) return;   // no slot of this tile is live
    __shared__ uint32_t base[256];          // running output offset per digit for this block
    __shared__ uint32_t wcnt[kWaves][256];  // per-wave digit counts, then per-wave offsets
    __shared__ uint32_t tot[256];
    const uint32_t tid = threadIdx.x, wave = tid >> 6;
    tot[tid] = totals[tid];
    for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    if (tid == 0) {   // exclusive scan of the 256 digit totals
        uint32_t run = 0;
        for (int d = 0; d < 256; ++d) { const uint32_t t = tot[d]; tot[d] = run; run += t; }
    }
    __syncthreads();
    base[tid] = tot[tid] + counts[(size_t)tid * nblocks + blockIdx.x];
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    for (int it = 0; it < kRsItems; ++it) {
        const uint32_t i = blockIdx.x * kSortTile + it * kRsThreads + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? keys_in[i] : 0u;
        const uint32_t val = valid ? (vals_in ? vals_in[i] : i) : 0u;
        const uint32_t d = (key >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot((d >> b) & 1u);
            same &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(same & lt);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(same);
        __syncthreads();
        {   // per digit: offsets of each wave, advance the running base
            uint32_t run = base[tid];
            for (int w = 0; w < kWaves; ++w) { const uint32_t c = wcnt[w][tid]; wcnt[w][tid] = run; run += c; }
            base[tid] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wcnt[wave][d] + rank;
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
        __syncthreads();
    }
}

hipError_t launch_radix_sort(OrderScratch &sc, const uint32_t *np, uint32_t n_max, int bits, uint32_t **perm_out,
                             hipStream_t s) {
    const uint32_t nblocks = (n_max + kSortTile - 1) / kSortTile;
    if (nblocks > sc.max_blocks) return hipErrorInvalidValue;
    int cur = 0;
    const uint32_t *vals_in = nullptr;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(kRsThreads), 0, s, sc.keys[cur], np, shift, sc.counts,
                           nblocks);
        hipLaunchKernelGGL(k_rs_scan_digit, dim3(256), dim3(kRsThreads), 0, s, sc.counts, nblocks, sc.totals);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(kRsThreads), 0, s, sc.keys[cur], vals_in,
                           sc.keys[cur ^ 1], sc.vals[cur ^ 1], np, shift, sc.counts, sc.totals, nblocks);
        vals_in = sc.vals[cur ^ 1];
        cur ^= 1;
    }
    *perm_out = sc.vals[cur];
    sc.sorted_keys = sc.keys[cur];
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Compaction: stable partition (active first) from wavefront ballots.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_compact_count(const uint32_t *status, const uint32_t *np,
                                                       uint32_t *block_alive) {
    __shared__ uint32_t wsum[4];
    const uint32_t n = *np;
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    const bool alive = i < n && status[i] == GC_ACTIVE;
    const uint64_t b = __ballot(alive);
    if ((threadIdx.x & 63u) == 0) wsum[threadIdx.x >> 6] = (uint32_t)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) block_alive[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// single workgroup: exclusive scan of the per-block counts, total -> n_active
__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t *v, uint32_t nb, uint32_t *n_active) {
    __shared__ uint32_t sh[1024];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t x = i < nb ? v[i] : 0u;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t t = threadIdx.x >= (uint32_t)off ? sh[threadIdx.x - off] : 0u;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) v[i] = carry + sh[threadIdx.x] - x;
        carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_active = carry;
}

__global__ __launch_bounds__(256) void k_compact_scatter(const uint32_t *status, const uint32_t *np,
                                                         const uint32_t *block_off, const uint32_t *n_active,
                                                         uint32_t *perm) {
    __shared__ uint32_t wsum[4];
    const uint32_t n = *np;
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    const bool valid = i < n;
    const bool alive = valid && status[i] == GC_ACTIVE;
    const uint64_t b = __ballot(alive);
    const uint32_t w = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) wsum[w] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t before = block_off[blockIdx.x];
    for (uint32_t q = 0; q < w; ++q) before += wsum[q];
    before += (uint32_t)__popcll(b & lanemask_lt());     // active slots before i
    if (valid) {
        const uint32_t pos = alive ? before : *n_active + (i - before);
        perm[pos] = i;
    }
}

hipError_t launch_compact(const SoA &st, const uint32_t *np, uint32_t n_max, OrderScratch &sc, uint32_t *n_active,
                          uint32_t **perm_out, hipStream_t s) {
    const uint32_t nb = (n_max + 255) / 256;
    if (nb == 0) return launch_fill_u32(n_active, 0u, 1, s);
    if (nb > 256u * sc.max_blocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_compact_count, dim3(nb), dim3(256), 0, s, st.status, np, sc.counts);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, sc.counts, nb, n_active);
    hipLaunchKernelGGL(k_compact_scatter, dim3(nb), dim3(256), 0, s, st.status, np, sc.counts, n_active, sc.vals[0]);
    *perm_out = sc.vals[0];
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <bool kWithComp>
__global__ void k_permute(SoA src, SoA dst, const uint32_t *perm, const uint32_t *np) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *np) return;
    const uint32_t j = perm[i];
#define P_(name) dst.name[i] = src.name[j];
    P_(r) P_(th) P_(ph) P_(u) P_(mu) P_(fr) P_(fth) P_(fph) P_(fu) P_(dtp) P_(s) P_(ell) P_(t)
    P_(k) P_(flags) P_(status) P_(step) P_(id) P_(ens) P_(gid) P_(birth)
    if (kWithComp) { P_(cr) P_(cth) P_(cph) P_(cu) P_(ct) }
#undef P_
}

hipError_t launch_permute(const SoA &src, const SoA &dst, const uint32_t *perm, const uint32_t *np, uint32_t n_max,
                          bool with_comp, hipStream_t s) {
    if (n_max == 0) return hipSuccess;
    const dim3 grid((n_max + 255) / 256);
    if (with_comp) hipLaunchKernelGGL(k_permute<true>, grid, dim3(256), 0, s, src, dst, perm, np);
    else hipLaunchKernelGGL(k_permute<false>, grid, dim3(256), 0, s, src, dst, perm, np);
    return hipGetLastError();
}

// Both state buffers hold identical data for the dead tail: slots past the
// live prefix are never permuted again.  After a permute, the particles that
// died since the last reorder (slots [*lo, *hi) of the new buffer) are copied
// back into the other buffer, which keeps the two in agreement on the tail.
__global__ void k_copy_range(SoA src, SoA dst, const uint32_t *lo, const uint32_t *hi, bool with_comp) {
    const uint32_t i = *lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *hi) return;
#define T_(name) dst.name[i] = src.name[i];
    T_(r) T_(th) T_(ph) T_(u) T_(mu) T_(fr) T_(fth) T_(fph) T_(fu) T_(dtp) T_(s) T_(ell) T_(t)
    T_(k) T_(flags) T_(status) T_(step) T_(id) T_(ens) T_(gid) T_(birth)
    if (with_comp) { T_(cr) T_(cth) T_(cph) T_(cu) T_(ct) }
#undef T_
}

hipError_t launch_copy_range(const SoA &src, const SoA &dst, const uint32_t *lo, const uint32_t *hi, uint32_t n_max,
                             bool with_comp, hipStream_t s) {
    if (n_max == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_range, dim3((n_max + 255) / 256), dim3(256), 0, s, src, dst, lo, hi, with_comp);
    return hipGetLastError();
}

__global__ void k_copy_count(uint32_t *dst, const uint32_t *src, volatile uint32_t *host_mirror, uint32_t *prev) {
    const uint32_t v = *src;
    if (prev) *prev = *dst;
    *dst = v;
    if (host_mirror) *host_mirror = v;
}

hipError_t launch_copy_count(uint32_t *dst, const uint32_t *src, volatile uint32_t *host_mirror, uint32_t *prev,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(1), 0, s, dst, src, host_mirror, prev);
    return hipGetLastError();
}

// Cell keys of the last sort in slot order: the sorted keys over the sorted
// prefix [0, *sorted_n), the inactive key past it.
__global__ void k_keys_out(const uint32_t *sorted_keys, const uint32_t *sorted_n, uint32_t dead_key, uint32_t n,
                           uint32_t *out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = i < *sorted_n ? sorted_keys[i] : dead_key;
}

hipError_t launch_keys_out(const uint32_t *sorted_keys, const uint32_t *sorted_n, uint32_t dead_key, uint32_t n,
                           uint32_t *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_keys_out, dim3((n + 255) / 256), dim3(256), 0, s, sorted_keys, sorted_n, dead_key, n, out);
    return hipGetLastError();
}

__global__ void k_set_count(uint32_t *p, uint32_t v) { *p = v; }

hipError_t launch_set_count(uint32_t *n_active, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, s, n_active, n);
    return hipGetLastError();
}

}  // namespace gc
