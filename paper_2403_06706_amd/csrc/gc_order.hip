// gc_order.hip -- particle reordering between chunks of steps.
//
//  * cell binning: key = field cell of the particle (optionally coarsened),
//    inactive particles get the largest key; LSD radix sort (8-bit digits) of
//    (key, slot) pairs; permute the state (for the grid push, only the
//    particles stopped since the last reorder: the push applies the
//    permutation to the others as it reads them).  Particles of one cell then
//    sit in consecutive lanes, so their trilinear gathers hit the same cache
//    lines.
//    The key kernel also counts the digits of every pass; each pass is then
//    one kernel that ranks its tile, finds the tile's offset per digit by
//    looking back over the tiles before it, and scatters.
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

__device__ __forceinline__ uint32_t cell_key(const SoA &st, const FieldDev &f, uint32_t i, int coarsen,
                                             uint32_t dead_key, bool &alive) {
    alive = st.status[i] == GC_ACTIVE;
    if (!alive) return dead_key;
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
    return (((uint32_t)fi >> coarsen) * nthc + ((uint32_t)fj >> coarsen)) * nphc + ((uint32_t)km >> coarsen);
}

// lanes of the wavefront whose valid digit equals this lane's
__device__ __forceinline__ uint64_t same_digit(uint32_t d, bool valid) {
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t bb = __ballot((d >> b) & 1u);
        same &= ((d >> b) & 1u) ? bb : ~bb;
    }
    return same;
}

// Keys of the live prefix, one sort tile per workgroup; the digit counts of
// every pass and the number of active particles are added to the sort state
// (which the reset at the end of the previous reorder left at zero).
__global__ __launch_bounds__(kRsThreads) void k_cell_keys(SoA st, FieldDev f, const uint32_t *np, int coarsen,
                                                         uint32_t dead_key, int passes, uint32_t *keys,
                                                         uint32_t *state) {
    __shared__ uint32_t h[kMaxPasses][256];
    __shared__ uint32_t wsum[kWaves];
    const uint32_t n = *np, tid = threadIdx.x;
    if (blockIdx.x * kSortTile >= n) return;   // tile past the live prefix (uniform)
    for (int p = 0; p < kMaxPasses; ++p) h[p][tid] = 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    uint32_t alive_n = 0;
    for (int it = 0; it < kRsItems; ++it) {
        const uint32_t i = blockIdx.x * kSortTile + it * kRsThreads + tid;
        const bool valid = i < n;
        bool alive = false;
        uint32_t key = 0;
        if (valid) {
            key = cell_key(st, f, i, coarsen, dead_key, alive);
            keys[i] = key;
        }
        alive_n += alive ? 1u : 0u;
        for (int p = 0; p < passes; ++p) {
            const uint32_t d = (key >> (8 * p)) & 255u;
            const uint64_t same = same_digit(d, valid);
            if (valid && (same & lt) == 0) atomicAdd(&h[p][d], (uint32_t)__popcll(same));
        }
    }
    for (int off = 32; off > 0; off >>= 1) alive_n += __shfl_xor(alive_n, off);
    if ((tid & 63u) == 0) wsum[tid >> 6] = alive_n;
    __syncthreads();
    for (int p = 0; p < passes; ++p)
        if (h[p][tid]) atomicAdd(&state[kStHist + p * 256 + tid], h[p][tid]);
    if (tid == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWaves; ++w) t += wsum[w];
        if (t) atomicAdd(&state[kStAlive], t);
    }
}

hipError_t launch_cell_keys(const SoA &st, const FieldDev &f, const uint32_t *np, uint32_t n_max, int coarsen,
                            uint32_t dead_key, int bits, OrderScratch &sc, uint32_t *n_active, hipStream_t s,
                            hipEvent_t start) {
    if (n_max == 0) {
        if (start) (void)hipEventRecord(start, s);
        return launch_fill_u32(n_active, 0u, 1, s);
    }
    const int passes = (bits + 7) / 8;
    const uint32_t nb = (n_max + kSortTile - 1) / kSortTile;
    if (passes > kMaxPasses || nb > sc.max_blocks) return hipErrorInvalidValue;
    launch_timed(k_cell_keys, dim3(nb), dim3(kRsThreads), s, start, nullptr, st, f, np, coarsen, dead_key, passes,
                 sc.keys[0], sc.state);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// LSD radix sort, one 8-bit digit per pass, one kernel per pass.  A workgroup
// takes the next tile in start order from a ticket counter, ranks its 2,048
// items stably (per wavefront by ballots, then across wavefronts and item
// rounds in LDS) and publishes its count per digit.  Its offset per digit
// among the tiles before it comes from looking back over their published
// words: an inclusive prefix ends the walk, an aggregate adds to it and the
// walk goes on.  A tile waits only for tiles that took their tickets before it
// and so are already running; each publishes its aggregate before it waits
// itself, so every wait ends.  Look-back words carry a tag (reorder epoch and
// pass), so words of earlier passes read as not yet published and the array
// never needs clearing; the tag repeats after 2^28 reorders.
// ---------------------------------------------------------------------------
constexpr uint32_t kFlagAgg = 1, kFlagPrefix = 2;
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ __forceinline__ unsigned long long look_word(uint32_t tag, uint32_t flag, uint32_t v) {
    return ((unsigned long long)(tag & 0x3FFFFFFFu) << 34) | ((unsigned long long)flag << 32) | v;
}

__global__ __launch_bounds__(kRsThreads) void k_rs_pass(const uint32_t *keys_in, const uint32_t *vals_in,
                                                       uint32_t *keys_out, uint32_t *vals_out, const uint32_t *np,
                                                       int pass, uint32_t *state, unsigned long long *look,
                                                       uint32_t *n_active) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t wcnt[kRsItems][kWaves][256];   // per (round, wave, digit): count, then offset in the tile
    __shared__ uint32_t s_base[256];
    const uint32_t tid = threadIdx.x, wave = tid >> 6;
    const uint32_t n = *np;
    // Only the first ceil(n / kSortTile) workgroups take tickets, so the tiles
    // of the live prefix are taken once each, in start order; the others leave
    // at once (workgroup 0 then publishes the active count of an empty prefix).
    if (blockIdx.x * kSortTile >= n) {
        if (pass == 0 && blockIdx.x == 0 && tid == 0) *n_active = state[kStAlive];
        return;
    }
    if (tid == 0) {
        s_tile = atomicAdd(&state[kStTicket + pass], 1u);
        if (pass == 0 && s_tile == 0) *n_active = state[kStAlive];
    }
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t tag = (state[kStEpoch] + 1u) * 4u + (uint32_t)pass;
    const int shift = 8 * pass;
#pragma unroll
    for (int it = 0; it < kRsItems; ++it)
        for (int w = 0; w < kWaves; ++w) wcnt[it][w][tid] = 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    uint32_t key[kRsItems], val[kRsItems], rank[kRsItems];
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const uint32_t i = tile * kSortTile + it * kRsThreads + tid;
        const bool valid = i < n;
        key[it] = valid ? keys_in[i] : 0xFFFFFFFFu;
        val[it] = valid ? (vals_in ? vals_in[i] : i) : 0u;
        const uint32_t d = (key[it] >> shift) & 255u;
        const uint64_t same = same_digit(d, valid);
        rank[it] = (uint32_t)__popcll(same & lt);
        if (valid && rank[it] == 0) wcnt[it][wave][d] = (uint32_t)__popcll(same);
    }
    __syncthreads();
    // thread tid owns digit tid: offsets of each (round, wave) within the tile
    uint32_t count = 0;
#pragma unroll
    for (int it = 0; it < kRsItems; ++it)
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = wcnt[it][w][tid];
            wcnt[it][w][tid] = count;
            count += c;
        }
    unsigned long long *mine = look + (size_t)tile * 256 + tid;
    uint32_t prefix = 0;
    if (tile == 0) {
        __hip_atomic_store(mine, look_word(tag, kFlagPrefix, count), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(mine, look_word(tag, kFlagAgg, count), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long want = (unsigned long long)(tag & 0x3FFFFFFFu);
        uint32_t j = tile - 1, spins = 0;
        for (;;) {
            const unsigned long long w =
                __hip_atomic_load(look + (size_t)j * 256 + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t flag = (uint32_t)(w >> 32) & 3u;
            if ((w >> 34) == want && flag != 0) {
                prefix += (uint32_t)w;
                if (flag == kFlagPrefix || j == 0) break;
                --j;
            } else if (++spins > kSpinLimit) {
                atomicOr(&state[kStError], 1u);   // reported by the next synchronizing call
                break;
            } else {
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __hip_atomic_store(mine, look_word(tag, kFlagPrefix, prefix + count), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    // global start of each digit: exclusive scan of this pass's digit totals
    const uint32_t tot = state[kStHist + pass * 256 + tid];
    s_base[tid] = tot;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t t = tid >= (uint32_t)off ? s_base[tid - off] : 0u;
        __syncthreads();
        s_base[tid] += t;
        __syncthreads();
    }
    const uint32_t start = s_base[tid] - tot + prefix;
    __syncthreads();
    s_base[tid] = start;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const uint32_t i = tile * kSortTile + it * kRsThreads + tid;
        if (i < n) {
            const uint32_t d = (key[it] >> shift) & 255u;
            const uint32_t pos = s_base[d] + wcnt[it][wave][d] + rank[it];
            if (pos < n) {   // always, with digit counts of these keys
                keys_out[pos] = key[it];
                vals_out[pos] = val[it];
            }
        }
    }
}

hipError_t launch_radix_sort(OrderScratch &sc, const uint32_t *np, uint32_t n_max, int bits, uint32_t *n_active,
                             uint32_t **perm_out, hipStream_t s) {
    const uint32_t nblocks = (n_max + kSortTile - 1) / kSortTile;
    const int passes = (bits + 7) / 8;
    if (nblocks > sc.max_blocks || passes > kMaxPasses) return hipErrorInvalidValue;
    int cur = 0;
    const uint32_t *vals_in = nullptr;
    for (int p = 0; p < passes && nblocks > 0; ++p) {
        hipLaunchKernelGGL(k_rs_pass, dim3(nblocks), dim3(kRsThreads), 0, s, sc.keys[cur], vals_in, sc.keys[cur ^ 1],
                           sc.vals[cur ^ 1], np, p, sc.state, sc.look, n_active);
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
                          uint32_t **perm_out, hipStream_t s, hipEvent_t start) {
    const uint32_t nb = (n_max + 255) / 256;
    if (nb == 0) {
        if (start) (void)hipEventRecord(start, s);
        return launch_fill_u32(n_active, 0u, 1, s);
    }
    if (nb > 256u * sc.max_blocks) return hipErrorInvalidValue;
    launch_timed(k_compact_count, dim3(nb), dim3(256), s, start, nullptr, st.status, np, sc.counts);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, sc.counts, nb, n_active);
    hipLaunchKernelGGL(k_compact_scatter, dim3(nb), dim3(256), 0, s, st.status, np, sc.counts, n_active, sc.vals[0]);
    *perm_out = sc.vals[0];
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <bool kWithComp>
__global__ void k_permute(SoA src, SoA dst, const uint32_t *perm, const uint32_t *lo, const uint32_t *hi) {
    const uint32_t i = (lo ? *lo : 0u) + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *hi) return;
    const uint32_t j = perm[i];
#define P_(name) dst.name[i] = src.name[j];
    P_(r) P_(th) P_(ph) P_(u) P_(mu) P_(fr) P_(fth) P_(fph) P_(fu) P_(dtp) P_(s) P_(ell) P_(t)
    P_(k) P_(flags) P_(status) P_(step) P_(id) P_(ens) P_(gid) P_(birth)
    if (kWithComp) { P_(cr) P_(cth) P_(cph) P_(cu) P_(ct) }
#undef P_
}

hipError_t launch_permute(const SoA &src, const SoA &dst, const uint32_t *perm, const uint32_t *lo,
                          const uint32_t *hi, uint32_t n_max, bool with_comp, hipStream_t s) {
    if (n_max == 0) return hipSuccess;
    const dim3 grid((n_max + 255) / 256);
    if (with_comp) hipLaunchKernelGGL(k_permute<true>, grid, dim3(256), 0, s, src, dst, perm, lo, hi);
    else hipLaunchKernelGGL(k_permute<false>, grid, dim3(256), 0, s, src, dst, perm, lo, hi);
    return hipGetLastError();
}

// Both state buffers hold identical data for the dead tail: slots past the
// live prefix are never permuted again.  After a permute, the particles that
// died since the last reorder (slots [*lo, *hi) of the new buffer) are copied
// back into the other buffer, which keeps the two in agreement on the tail.
__global__ __launch_bounds__(256) void k_copy_range(SoA src, SoA dst, const uint32_t *lo, const uint32_t *hi,
                                                    bool with_comp, unsigned long long *dead) {
    __shared__ unsigned long long part[4][6];
    const uint32_t b0 = *lo + blockIdx.x * blockDim.x, end = *hi;
    if (b0 >= end) return;                        // workgroup past the range (uniform)
    const uint32_t i = b0 + threadIdx.x;
    const bool in = i < end;
    uint32_t status = 0xFFFFFFFFu;
    unsigned long long k = 0, step = 0;
    if (in) {
#define T_(name) dst.name[i] = src.name[i];
        T_(r) T_(th) T_(ph) T_(u) T_(mu) T_(fr) T_(fth) T_(fph) T_(fu) T_(dtp) T_(s) T_(ell) T_(t)
        T_(k) T_(flags) T_(status) T_(step) T_(id) T_(ens) T_(gid) T_(birth)
        if (with_comp) { T_(cr) T_(cth) T_(cph) T_(cu) T_(ct) }
#undef T_
        status = src.status[i];
        k = src.k[i];
        step = src.step[i];
    }
    if (!dead) return;
    // the slots leave the live prefix for good: their sums join dead[], one
    // atomic per sum and workgroup
    unsigned long long v[6];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (unsigned long long)__popcll(__ballot(in && status == (uint32_t)q));
    for (int off = 32; off > 0; off >>= 1) {
        k += __shfl_xor(k, off);
        step += __shfl_xor(step, off);
    }
    v[4] = k;
    v[5] = step;
    const uint32_t wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0)
        for (int q = 0; q < 6; ++q) part[wave][q] = v[q];
    __syncthreads();
    if (threadIdx.x < 6) {
        const unsigned long long t = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] +
                                     part[3][threadIdx.x];
        if (t) atomicAdd(&dead[threadIdx.x], t);
    }
}

hipError_t launch_copy_range(const SoA &src, const SoA &dst, const uint32_t *lo, const uint32_t *hi, uint32_t n_max,
                             bool with_comp, unsigned long long *dead, hipStream_t s) {
    if (n_max == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_range, dim3((n_max + 255) / 256), dim3(256), 0, s, src, dst, lo, hi, with_comp, dead);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy_count(uint32_t *dst, const uint32_t *src,
                                                    volatile uint32_t *host_mirror, uint32_t *prev,
                                                    uint32_t *state) {
    const uint32_t tid = threadIdx.x;
    if (tid == 0) {
        const uint32_t v = *src;
        if (prev) *prev = *dst;
        *dst = v;
        if (host_mirror) *host_mirror = v;
        state[kStEpoch] += 1u;
        state[kStAlive] = 0;
    }
    for (uint32_t i = tid; i < kMaxPasses * 256; i += 256) state[kStHist + i] = 0;
    if (tid < kMaxPasses) state[kStTicket + tid] = 0;
}

hipError_t launch_copy_count(uint32_t *dst, const uint32_t *src, volatile uint32_t *host_mirror, uint32_t *prev,
                             uint32_t *state, hipStream_t s, hipEvent_t stop) {
    launch_timed(k_copy_count, dim3(1), dim3(256), s, nullptr, stop, dst, src, host_mirror, prev, state);
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

__global__ void k_reset_bound(uint32_t *n_bound, uint32_t n, unsigned long long *dead) {
    if (threadIdx.x == 0) *n_bound = n;
    if (threadIdx.x < 6) dead[threadIdx.x] = 0;
}

hipError_t launch_reset_bound(uint32_t *n_bound, uint32_t n, unsigned long long *dead, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_bound, dim3(1), dim3(64), 0, s, n_bound, n, dead);
    return hipGetLastError();
}

hipError_t launch_set_count(uint32_t *n_active, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, s, n_active, n);
    return hipGetLastError();
}

}  // namespace gc
