// gc_launch.h -- host-side launchers of the kernels (defined in the .hip files).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "gc_internal.h"

namespace gc {

struct MomDev {
    int32_t n_rbins, n_mubins, n_agebins, n_ebins, min_collisions, total;
    uint32_t min_birth;
    int32_t accumulate;
    double r_lo, r_hi, sel_r_lo, sel_r_hi, age_lo, age_hi, age_max, e_lo, e_hi, e_unit, len_unit;
};

// Timing events attached to the dispatches of a kernel sequence: start takes the
// start time of its first kernel, stop the end time of its last.  Attached to
// the dispatch packets they add no marker packets to the queue (hipEventRecord
// would, each costing the queue several microseconds).  Null: not timed.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

// A plain launch without events (the form stream capture records), else the
// launch with the events attached to its dispatch.
template <typename... KArgs, typename... Args>
inline void launch_timed(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t s, hipEvent_t start,
                         hipEvent_t stop, Args... args) {
    if (start || stop)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, start, stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// push (gc_push.hip); form: 0 throughput, 1 all pairs of a gather in flight,
// 2 four lanes per particle (the last two for few active particles)
hipError_t launch_push(const PushArgs &a, int precision, int block, bool persistent, int form, int grid_blocks,
                       hipStream_t s, LaunchEvents ev = {});

// gather ceiling (gc_probe.hip): sink[slot] for every slot below *a.n_active
hipError_t launch_gather_probe(const PushArgs &a, double *sink, int block, hipStream_t s);

// injection, state copies, fills (gc_kernels.hip); moments (gc_moments.hip)
hipError_t launch_inject(const SoA &st, const FieldDev &f, const EnsDev &e, uint32_t n0, uint32_t n,
                         uint32_t first_id, uint32_t eidx, hipStream_t s);
// n_scan (device, nullable): only slots [0, *n_scan) are read, and dead (device,
// nullable) holds the sums [0..5] over the slots past it (particles per status,
// collision counts, steps), added to out; else all n slots are read
hipError_t launch_moments(const SoA &st, const FieldDev &f, const EnsDev *ens, uint32_t n, const MomDev &m,
                          unsigned long long *out, const uint32_t *n_scan, const unsigned long long *dead,
                          hipStream_t s);
hipError_t launch_state_out(const SoA &st, const gc_state_view &dst, uint32_t n, hipStream_t s);
hipError_t launch_state_in(const SoA &st, const gc_state_view &src, uint32_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, size_t n, hipStream_t s);
hipError_t launch_copy_probe(void *dst, const void *src, size_t n_bytes, hipStream_t s);
hipError_t launch_pack_field(const double *src, void *dst, int nr, int nth, int nph, int dtype, int records,
                             const float *inv_scale, hipStream_t s);

// reordering (gc_order.hip)
constexpr int kSortTile = 2048;     // items per radix-sort tile (one workgroup)
constexpr int kMaxPasses = 4;       // 8-bit digits of a 32-bit key
// Sort state (uint32 words), zero when a context allocates it; the reset at the
// end of every reorder clears the counts and tickets and advances the epoch.
constexpr int kStHist = 0;                          // [kMaxPasses][256] digit counts of the keys
constexpr int kStAlive = kStHist + kMaxPasses * 256; // active particles among the keys
constexpr int kStTicket = kStAlive + 1;              // [kMaxPasses] next tile of each pass
constexpr int kStEpoch = kStTicket + kMaxPasses;     // reorders completed (look-back tags)
constexpr int kStError = kStEpoch + 1;               // nonzero: a look-back did not complete
constexpr int kStWords = 1088;
static_assert(kStError < kStWords, "sort state layout");
struct OrderScratch {
    uint32_t *keys[2];
    uint32_t *vals[2];
    uint32_t *counts;            // [256 * max_blocks] per-block active counts of the compaction
    uint32_t *state;             // [kStWords]
    unsigned long long *look;    // [max_blocks][256] look-back words of the radix sort
    uint32_t max_blocks;         // sort tiles the buffers hold
    uint32_t *sorted_keys;       // keys[0] or keys[1]: the keys in slot order after the last radix sort
};
// Reorder kernels act on the live prefix [0, *np) of the slots (np in device
// memory); n_max (host) is an upper bound used to size the grids.
// cell keys of the live prefix into sc.keys[0], with the digit counts of every
// pass of a bits-wide sort and the active count added to sc.state
hipError_t launch_cell_keys(const SoA &st, const FieldDev &f, const uint32_t *np, uint32_t n_max, int coarsen,
                            uint32_t dead_key, int bits, OrderScratch &sc, uint32_t *n_active, hipStream_t s,
                            hipEvent_t start = nullptr);
// stable sort of (sc.keys[0], slot) by the low bits of the keys from launch_cell_keys;
// *n_active = the active count; perm_out: sorted slots
hipError_t launch_radix_sort(OrderScratch &sc, const uint32_t *np, uint32_t n_max, int bits, uint32_t *n_active,
                             uint32_t **perm_out, hipStream_t s);
hipError_t launch_compact(const SoA &st, const uint32_t *np, uint32_t n_max, OrderScratch &sc, uint32_t *n_active,
                          uint32_t **perm_out, hipStream_t s, hipEvent_t start = nullptr);
// dst[i] = src[perm[i]] for i in [*lo, *hi) (lo null: from 0)
hipError_t launch_permute(const SoA &src, const SoA &dst, const uint32_t *perm, const uint32_t *lo,
                          const uint32_t *hi, uint32_t n_max, bool with_comp, hipStream_t s);
// dst[i] = src[i] for i in [*lo, *hi); with dead set, the per-status counts,
// collision counts and steps of those slots are added to dead[0..5]
hipError_t launch_copy_range(const SoA &src, const SoA &dst, const uint32_t *lo, const uint32_t *hi, uint32_t n_max,
                             bool with_comp, unsigned long long *dead, hipStream_t s);
// *n_bound = n and dead[0..5] = 0: the live prefix is every slot again
hipError_t launch_reset_bound(uint32_t *n_bound, uint32_t n, unsigned long long *dead, hipStream_t s);
// *dst = *src; also *host_mirror = *src when host_mirror (host-coherent pinned memory) is set,
// and *prev = the old *dst when prev is set; then resets the sort state for the next reorder
hipError_t launch_copy_count(uint32_t *dst, const uint32_t *src, volatile uint32_t *host_mirror, uint32_t *prev,
                             uint32_t *sort_state, hipStream_t s, hipEvent_t stop = nullptr);
// out[i] = i < *sorted_n ? sorted_keys[i] : dead_key for i < n
hipError_t launch_keys_out(const uint32_t *sorted_keys, const uint32_t *sorted_n, uint32_t dead_key, uint32_t n,
                           uint32_t *out, hipStream_t s);
hipError_t launch_set_count(uint32_t *n_active, uint32_t n, hipStream_t s);

}  // namespace gc
