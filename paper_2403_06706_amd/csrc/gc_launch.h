// gc_launch.h -- host-side launchers of the kernels (defined in the .hip files).
#pragma once
#include <hip/hip_runtime.h>

#include "gc_internal.h"

namespace gc {

struct MomDev {
    int32_t n_rbins, n_mubins, n_agebins, n_ebins, min_collisions, total;
    uint32_t min_birth;
    int32_t accumulate;
    double r_lo, r_hi, sel_r_lo, sel_r_hi, age_lo, age_hi, age_max, e_lo, e_hi, e_unit, len_unit;
};

// push (gc_push.hip); form: 0 throughput, 1 all pairs of a gather in flight,
// 2 four lanes per particle (the last two for few active particles)
hipError_t launch_push(const PushArgs &a, int precision, int block, bool persistent, int form, int grid_blocks,
                       hipStream_t s);

// gather ceiling (gc_probe.hip): sink[slot] for every slot below *a.n_active
hipError_t launch_gather_probe(const PushArgs &a, double *sink, int block, hipStream_t s);

// injection, state copies, fills (gc_kernels.hip); moments (gc_moments.hip)
hipError_t launch_inject(const SoA &st, const FieldDev &f, const EnsDev &e, uint32_t n0, uint32_t n,
                         uint32_t first_id, uint32_t eidx, hipStream_t s);
hipError_t launch_moments(const SoA &st, const FieldDev &f, const EnsDev *ens, uint32_t n, const MomDev &m,
                          unsigned long long *out, hipStream_t s);
hipError_t launch_state_out(const SoA &st, const gc_state_view &dst, uint32_t n, hipStream_t s);
hipError_t launch_state_in(const SoA &st, const gc_state_view &src, uint32_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, size_t n, hipStream_t s);
hipError_t launch_copy_probe(void *dst, const void *src, size_t n_bytes, hipStream_t s);
hipError_t launch_pack_field(const double *src, void *dst, int nr, int nth, int nph, int dtype, int records,
                             const float *inv_scale, hipStream_t s);

// reordering (gc_order.hip)
struct OrderScratch {
    uint32_t *keys[2];
    uint32_t *vals[2];
    uint32_t *counts;      // [256][max_blocks] radix histograms, or per-block alive counts
    uint32_t *totals;      // [256]
    uint32_t *block_alive; // [n / 256] active particles per 256-slot block
    uint32_t max_blocks;
    uint32_t *sorted_keys; // keys[0] or keys[1]: the keys in slot order after the last radix sort
};
constexpr int kSortTile = 2048;     // items per radix-sort block
// Reorder kernels act on the live prefix [0, *np) of the slots (np in device
// memory); n_max (host) is an upper bound used to size the grids.
hipError_t launch_cell_keys(const SoA &st, const FieldDev &f, const uint32_t *np, uint32_t n_max, int coarsen,
                            uint32_t dead_key, uint32_t *keys, uint32_t *block_alive, uint32_t *n_active,
                            hipStream_t s);
hipError_t launch_radix_sort(OrderScratch &sc, const uint32_t *np, uint32_t n_max, int bits, uint32_t **perm_out,
                             hipStream_t s);
hipError_t launch_compact(const SoA &st, const uint32_t *np, uint32_t n_max, OrderScratch &sc, uint32_t *n_active,
                          uint32_t **perm_out, hipStream_t s);
hipError_t launch_permute(const SoA &src, const SoA &dst, const uint32_t *perm, const uint32_t *np, uint32_t n_max,
                          bool with_comp, hipStream_t s);
hipError_t launch_copy_range(const SoA &src, const SoA &dst, const uint32_t *lo, const uint32_t *hi, uint32_t n_max,
                             bool with_comp, hipStream_t s);
// *dst = *src; also *host_mirror = *src when host_mirror (host-coherent pinned memory) is set,
// and *prev = the old *dst when prev is set
hipError_t launch_copy_count(uint32_t *dst, const uint32_t *src, volatile uint32_t *host_mirror, uint32_t *prev,
                             hipStream_t s);
// out[i] = i < *sorted_n ? sorted_keys[i] : dead_key for i < n
hipError_t launch_keys_out(const uint32_t *sorted_keys, const uint32_t *sorted_n, uint32_t dead_key, uint32_t n,
                           uint32_t *out, hipStream_t s);
hipError_t launch_set_count(uint32_t *n_active, uint32_t n, hipStream_t s);

}  // namespace gc
