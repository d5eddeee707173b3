// gc_api.cpp -- host implementation of the C ABI declared in gcpush.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "gc_internal.h"
#include "gc_launch.h"
#include "gc_mlp.h"
#include "gc_mlp_launch.h"
#include "gcpush.h"

using namespace gc;

constexpr int kPushForms = 3;

struct GraphKey {
    double dt = 0;
    int64_t n_steps = -1;
    uint64_t n = 0;
    const void *state = nullptr;    // buffer holding the state at capture (eager reorders swap buffers)
    gc_options opt{};
};

// Training workspace of the neural field for some number of rows (carve_ws).
struct TrainWs {
    __bf16 *H = nullptr, *dZ = nullptr;                  // H: activations H0..H6, [7][rows][128]
    float *Z = nullptr, *Y = nullptr, *dY = nullptr;     // Z: pre-activations [6][rows][128]
    float *dH = nullptr, *part = nullptr;                // part: split-K and column-sum partials
    double *loss_part = nullptr;
};

// Neural field: FP32 master parameters (padded device layout), Adam moments,
// gradient and the BF16 copies used by the matrix-core products; training
// workspace sized for ws_rows rows.
struct MlpState {
    bool set = false;
    MlpArgs args{};
    void *mem = nullptr;
    float *p = nullptr, *mo = nullptr, *ve = nullptr, *g = nullptr;
    __bf16 *W = nullptr, *WT = nullptr, *Wo = nullptr;   // natural order (training)
    __bf16 *We = nullptr, *Woe = nullptr;                 // evaluation order (mlp_perm)
    void *ws = nullptr;
    int64_t ws_rows = 0;
    TrainWs w{};                                         // carved from ws
};

struct gc_ctx {
    gc_options opt{};
    hipStream_t stream = nullptr;
    std::string err;
    int n_cus = 256;
    // field
    bool have_field = false;
    void *field_buf = nullptr;
    void *field_rec_buf = nullptr;    // node records of the field (quad form; FP32/FP64 stores)
    FieldDev f{};
    FieldDev *f_dev = nullptr;        // device copy of f
    FieldDev fx{};                    // the extra node array of the full Eqs. 1-2 (data NULL if none)
    void *extra_buf = nullptr;
    // ensembles
    std::vector<EnsDev> ens_host;
    std::vector<char> ens_set;
    EnsDev *ens_dev = nullptr;
    bool any_rebirth = false;         // some ensemble has rebirth_steps > 0
    bool any_wind = false;            // some ensemble scatters in the wind frame
    // particles (A is current, B the target of a reorder's permutation)
    uint64_t n = 0, cap = 0;
    void *soa_mem[2] = {nullptr, nullptr};
    SoA A{}, B{};
    OrderScratch sc{};
    void *scratch_mem = nullptr;
    uint32_t *n_active = nullptr;
    uint32_t *queue = nullptr;
    uint32_t *n_bound = nullptr;      // live prefix: slots at or past it hold no active particle
    uint32_t *sorted_n = nullptr;     // length of the prefix the last reorder sorted
    unsigned long long *dead = nullptr;   // [6] sums over the slots past n_bound (moments [0..5])
    bool bound_dirty = true;          // the bound must be reset to n before the next reorder
    bool order_known = false;         // a reorder ran since the particle set last changed
    bool keys_known = false;          // ... and it was a cell binning (its keys are in sc.sorted_keys)
    uint32_t sorted_dead = 0;         // the inactive key of that binning
    // a reorder whose permutation the next push applies (grid field source):
    // the permutation, the order kind, and the reorder's timing events
    uint32_t *pend_perm = nullptr;
    int pend_order = 0;
    hipEvent_t pend_e0 = nullptr, pend_e1 = nullptr;
    unsigned long long *steps = nullptr;       // [kPushForms] active particle-steps by push form
    uint32_t *log = nullptr;
    volatile uint32_t *count_host = nullptr;   // live count of the latest completed reorder (pinned)
    bool capturing = false;
    int tail_skip = 0;                         // reorders still to skip in the tail
    hipEvent_t ahead[4] = {nullptr, nullptr, nullptr, nullptr};   // ends of the last chunks issued
    int ahead_pos = 0;
    // timing
    struct PushEv { hipEvent_t e0, e1; int form; };
    std::vector<PushEv> ev_push;
    // a reorder's span; with p0, p1 set the span holds that push, not counted
    struct ReorderEv { hipEvent_t e0, e1, p0, p1; };
    std::vector<ReorderEv> ev_reorder;
    std::vector<hipEvent_t> ev_pool;   // recorded and read events, ready for reuse
    // graph
    hipGraphExec_t gexec = nullptr;
    GraphKey gkey{};
    // neural field
    MlpState mlp;
};

namespace {

gc_status fail(gc_ctx *c, gc_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(ctx, GC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

bool valid_block(int b) { return b == 64 || b == 128 || b == 256; }

void scratch_init(int device);   // the static training workspace (below), once per device

gc_status check_options(gc_ctx *ctx, const gc_options *o) {
    if (o->precision < GC_PREC_F64 || o->precision > GC_PREC_F32_KAHAN)
        return fail(ctx, GC_EINVAL, "unknown precision %d", o->precision);
    if (o->order < GC_ORDER_NONE || o->order > GC_ORDER_BIN) return fail(ctx, GC_EINVAL, "unknown order %d", o->order);
    if (o->chunk_steps <= 0) return fail(ctx, GC_EINVAL, "chunk_steps must be > 0");
    if (o->bin_coarsen < 0 || o->bin_coarsen > 6) return fail(ctx, GC_EINVAL, "bin_coarsen must be in [0, 6]");
    if (!valid_block(o->block_size)) return fail(ctx, GC_EINVAL, "block_size must be 64, 128 or 256");
    if (o->persistent && (o->tile <= 0 || o->tile % o->block_size != 0))
        return fail(ctx, GC_EINVAL, "tile must be a positive multiple of block_size");
    if (o->log_depth < 0 || o->log_depth > 4096) return fail(ctx, GC_EINVAL, "log_depth must be in [0, 4096]");
    if (o->timing < 0 || o->timing > 2) return fail(ctx, GC_EINVAL, "timing must be 0, 1 or 2");
    if (o->field_source != GC_SOURCE_GRID && o->field_source != GC_SOURCE_MLP)
        return fail(ctx, GC_EINVAL, "unknown field_source %d", o->field_source);
    if (o->tail_threshold < 0) return fail(ctx, GC_EINVAL, "tail_threshold must be >= 0");
    if (!o->dev_alloc != !o->dev_free) return fail(ctx, GC_EINVAL, "dev_alloc and dev_free must be given together");
    return GC_OK;
}

// carve one allocation into the SoA arrays
void carve(void *mem, uint64_t cap, SoA &s) {
    double *d = static_cast<double *>(mem);
    double **dp[kNumDoubleArrays] = {&s.r, &s.th, &s.ph, &s.u, &s.mu, &s.fr, &s.fth, &s.fph, &s.fu,
                                     &s.dtp, &s.s, &s.ell, &s.t, &s.cr, &s.cth, &s.cph, &s.cu, &s.ct};
    for (int i = 0; i < kNumDoubleArrays; ++i) *dp[i] = d + (size_t)i * cap;
    uint32_t *u = reinterpret_cast<uint32_t *>(d + (size_t)kNumDoubleArrays * cap);
    uint32_t **up[kNumU32Arrays] = {&s.k, &s.flags, &s.status, &s.step, &s.id, &s.ens, &s.gid, &s.birth};
    for (int i = 0; i < kNumU32Arrays; ++i) *up[i] = u + (size_t)i * cap;
}

size_t soa_bytes(uint64_t cap) { return (size_t)cap * (kNumDoubleArrays * 8 + kNumU32Arrays * 4); }

// Device memory of the context: the caller's allocator when one was given at
// creation, else hipMalloc / hipFree.
hipError_t dalloc(gc_ctx *ctx, void **p, size_t bytes) {
    if (ctx->opt.dev_alloc) {
        *p = ctx->opt.dev_alloc(bytes, ctx->opt.alloc_user);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

void dfree(gc_ctx *ctx, void *p) {
    if (!p) return;
    if (ctx->opt.dev_free) ctx->opt.dev_free(p, ctx->opt.alloc_user);
    else (void)hipFree(p);
}

gc_status reserve(gc_ctx *ctx, uint64_t need) {
    if (need <= ctx->cap) return GC_OK;
    if (need > 0xFFFFFFF0ull) return fail(ctx, GC_EINVAL, "too many particles (%llu)", (unsigned long long)need);
    uint64_t cap = std::max<uint64_t>({need, ctx->cap * 2, 1024});
    cap = (cap + 2047) & ~uint64_t(2047);
    void *m[2] = {nullptr, nullptr};
    for (int i = 0; i < 2; ++i)
        if (dalloc(ctx, (void **)&m[i], soa_bytes(cap)) != hipSuccess) {
            if (m[0]) dfree(ctx, m[0]);
            return fail(ctx, GC_ENOMEM, "cannot allocate particle state for %llu particles", (unsigned long long)cap);
        }
    SoA na{}, nb{};
    carve(m[0], cap, na);
    carve(m[1], cap, nb);
    const uint32_t max_blocks = (uint32_t)((cap + kSortTile - 1) / kSortTile);
    const size_t look_bytes = (size_t)max_blocks * 256 * sizeof(unsigned long long);
    const size_t sort_bytes = look_bytes + (size_t)cap * 4 * 4 + (size_t)256 * max_blocks * 4 + kStWords * 4;
    void *sm = nullptr;
    if (dalloc(ctx, (void **)&sm, sort_bytes) != hipSuccess) {
        dfree(ctx, m[0]);
        dfree(ctx, m[1]);
        return fail(ctx, GC_ENOMEM, "cannot allocate sort scratch");
    }
    uint32_t *log = nullptr;
    if (ctx->opt.log_depth > 0 &&
        dalloc(ctx, (void **)&log, (size_t)cap * ctx->opt.log_depth * sizeof(uint32_t)) != hipSuccess) {
        dfree(ctx, m[0]);
        dfree(ctx, m[1]);
        dfree(ctx, sm);
        return fail(ctx, GC_ENOMEM, "cannot allocate collision log");
    }
    hipStream_t s = ctx->stream;
    // a failing device call releases the new buffers (the old state stays)
    auto release_new = [&]() {
        (void)hipStreamSynchronize(s);
        dfree(ctx, m[0]);
        dfree(ctx, m[1]);
        dfree(ctx, sm);
        dfree(ctx, log);
    };
#define RESERVE_CHK(expr)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) {                                                                        \
            release_new();                                                                             \
            return fail(ctx, GC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));                      \
        }                                                                                              \
    } while (0)
    if (log) RESERVE_CHK(launch_fill_u32(log, 0xFFFFFFFFu, (size_t)cap * ctx->opt.log_depth, s));
    // look-back words and sort state start at zero (never a valid look-back tag)
    RESERVE_CHK(launch_fill_u32(static_cast<uint32_t *>(sm), 0u, sort_bytes / 4, s));
    if (ctx->n > 0) {
        // keep the current state (and log) of the first n slots
        double **src_d[kNumDoubleArrays] = {&ctx->A.r, &ctx->A.th, &ctx->A.ph, &ctx->A.u, &ctx->A.mu, &ctx->A.fr,
                                            &ctx->A.fth, &ctx->A.fph, &ctx->A.fu, &ctx->A.dtp, &ctx->A.s, &ctx->A.ell,
                                            &ctx->A.t, &ctx->A.cr, &ctx->A.cth, &ctx->A.cph, &ctx->A.cu, &ctx->A.ct};
        double **dst_d[kNumDoubleArrays] = {&na.r, &na.th, &na.ph, &na.u, &na.mu, &na.fr, &na.fth, &na.fph, &na.fu,
                                            &na.dtp, &na.s, &na.ell, &na.t, &na.cr, &na.cth, &na.cph, &na.cu, &na.ct};
        for (int i = 0; i < kNumDoubleArrays; ++i)
            RESERVE_CHK(hipMemcpyAsync(*dst_d[i], *src_d[i], ctx->n * 8, hipMemcpyDeviceToDevice, s));
        uint32_t **src_u[kNumU32Arrays] = {&ctx->A.k, &ctx->A.flags, &ctx->A.status, &ctx->A.step,
                                           &ctx->A.id, &ctx->A.ens, &ctx->A.gid, &ctx->A.birth};
        uint32_t **dst_u[kNumU32Arrays] = {&na.k, &na.flags, &na.status, &na.step, &na.id, &na.ens, &na.gid,
                                           &na.birth};
        for (int i = 0; i < kNumU32Arrays; ++i)
            RESERVE_CHK(hipMemcpyAsync(*dst_u[i], *src_u[i], ctx->n * 4, hipMemcpyDeviceToDevice, s));
        if (log && ctx->log)
            RESERVE_CHK(hipMemcpyAsync(log, ctx->log, ctx->n * ctx->opt.log_depth * 4, hipMemcpyDeviceToDevice, s));
    }
    RESERVE_CHK(hipStreamSynchronize(s));
#undef RESERVE_CHK
    for (int i = 0; i < 2; ++i)
        if (ctx->soa_mem[i]) dfree(ctx, ctx->soa_mem[i]);
    if (ctx->scratch_mem) dfree(ctx, ctx->scratch_mem);
    if (ctx->log) dfree(ctx, ctx->log);
    ctx->soa_mem[0] = m[0];
    ctx->soa_mem[1] = m[1];
    ctx->A = na;
    ctx->B = nb;
    ctx->scratch_mem = sm;
    ctx->sc.look = static_cast<unsigned long long *>(sm);
    uint32_t *p = reinterpret_cast<uint32_t *>(static_cast<char *>(sm) + look_bytes);
    ctx->sc.keys[0] = p;
    ctx->sc.keys[1] = p + cap;
    ctx->sc.vals[0] = p + 2 * cap;
    ctx->sc.vals[1] = p + 3 * cap;
    ctx->sc.counts = p + 4 * cap;
    ctx->sc.state = ctx->sc.counts + (size_t)256 * max_blocks;
    ctx->sc.max_blocks = max_blocks;
    ctx->sc.sorted_keys = ctx->sc.keys[0];
    ctx->log = log;
    ctx->cap = cap;
    ctx->bound_dirty = true;
    ctx->order_known = ctx->keys_known = false;
    if (ctx->gexec) {
        (void)hipGraphExecDestroy(ctx->gexec);
        ctx->gexec = nullptr;
    }
    return GC_OK;
}

hipEvent_t take_event(gc_ctx *ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

uint32_t bits_for(uint32_t max_key) {
    uint32_t b = 1;
    while (b < 32 && (max_key >> b) != 0) ++b;
    return b;
}

// Tail of a run (eager advance only): once the live count read back from an
// earlier reorder is below tail_threshold, the machine is far from full and the
// push is bound by each wavefront's chain of dependent memory round trips.
// Then the push takes a latency form (all loads of a gather in flight; below
// threshold / kQuadShare, four lanes per particle), and the reorder runs
// only every kTailReorderEvery chunks (particles cross about two cells per 64
// steps, so the cell order decays slowly, while a reorder costs a fixed ~80 us
// of launches).  No choice changes any particle's trajectory.
constexpr int kTailReorderEvery = 8;
// The live count read back is only as fresh as the host's lead over the
// device: with the tail policy on, the host issues a chunk only once the chunk
// issued kAhead chunks earlier has finished (enough queued work to hide the
// launches, little enough for the count to follow the run).
constexpr int kAhead = 3;

uint32_t seen_count(const gc_ctx *ctx) {
    if (ctx->opt.tail_threshold <= 0 || ctx->capturing || !ctx->count_host) return 0xFFFFFFFFu;
    return *ctx->count_host;
}

bool tail_mode(const gc_ctx *ctx) {
    const uint32_t seen = seen_count(ctx);
    return seen != 0xFFFFFFFFu && seen < (uint32_t)ctx->opt.tail_threshold;
}

int push_form(const gc_ctx *ctx) {
    const uint32_t seen = seen_count(ctx);
    if (seen == 0xFFFFFFFFu || seen >= (uint32_t)ctx->opt.tail_threshold) return 0;
    return seen < (uint32_t)ctx->opt.tail_threshold / kQuadShare ? 2 : 1;
}

gc_status finish_reorder(gc_ctx *ctx, int order, hipEvent_t e0, hipEvent_t e1, hipEvent_t p0, hipEvent_t p1);

gc_status reorder(gc_ctx *ctx, bool timed, int order) {
    hipStream_t s = ctx->stream;
    const uint32_t n = (uint32_t)ctx->n;
    if (ctx->pend_perm)
        return fail(ctx, GC_ESTATE, "an earlier advance failed between a reorder and its push: "
                                    "reload the state (gc_set_state) or destroy the context");
    if (order == GC_ORDER_NONE) {
        HIPCHK(launch_set_count(ctx->n_active, n, s));
        ctx->bound_dirty = true;    // active particles may sit anywhere until the next reorder
        ctx->order_known = ctx->keys_known = false;
        return GC_OK;
    }
    if (ctx->bound_dirty) {
        HIPCHK(launch_reset_bound(ctx->n_bound, n, ctx->dead, s));
        ctx->bound_dirty = false;
    }
    // timed from the start of the first reorder kernel to the end of the last
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        e0 = take_event(ctx);
        e1 = take_event(ctx);
    }
    const bool comp = ctx->opt.precision == GC_PREC_F32_KAHAN;
    uint32_t *perm = nullptr;
    if (order == GC_ORDER_COMPACT) {
        HIPCHK(launch_compact(ctx->A, ctx->n_bound, n, ctx->sc, ctx->n_active, &perm, s, e0));
    } else {
        const int c = ctx->opt.bin_coarsen;
        const uint32_t nrc = ((uint32_t)ctx->f.nr + (1u << c) - 1) >> c;
        const uint32_t nthc = ((uint32_t)ctx->f.nth + (1u << c) - 1) >> c;
        const uint32_t nphc = ((uint32_t)ctx->f.nph + (1u << c) - 1) >> c;
        const uint32_t dead = nrc * nthc * nphc;
        ctx->sorted_dead = dead;
        const int bits = (int)bits_for(dead);
        HIPCHK(launch_cell_keys(ctx->A, ctx->f, ctx->n_bound, n, c, dead, bits, ctx->sc, ctx->n_active, s, e0));
        HIPCHK(launch_radix_sort(ctx->sc, ctx->n_bound, n, bits, ctx->n_active, &perm, s));
    }
    if (ctx->opt.field_source == GC_SOURCE_GRID) {
        // The grid push applies the permutation itself (it reads every active
        // particle from A through perm and writes it to B): here only the
        // particles stopped since the last reorder, slots [n_active, n_bound)
        // of the new order, move; the push ends the reorder.
        HIPCHK(launch_permute(ctx->A, ctx->B, perm, ctx->n_active, ctx->n_bound, n, comp, s));
        ctx->pend_perm = perm;
        ctx->pend_order = order;
        ctx->pend_e0 = e0;
        ctx->pend_e1 = e1;
        return GC_OK;
    }
    HIPCHK(launch_permute(ctx->A, ctx->B, perm, nullptr, ctx->n_bound, n, comp, s));
    return finish_reorder(ctx, order, e0, e1, nullptr, nullptr);
}

// The end of a reorder, once B holds the permuted state: the particles stopped
// since the last reorder, slots [n_active, n_bound) of B, are copied to A too
// (both buffers keep the same slots past the live prefix), the live prefix
// shrinks to the active count, and B becomes the current buffer.  e0, e1: the
// reorder's timing events (e1 attached here); p0, p1: those of a push between
// them that applied the permutation.
gc_status finish_reorder(gc_ctx *ctx, int order, hipEvent_t e0, hipEvent_t e1, hipEvent_t p0, hipEvent_t p1) {
    hipStream_t s = ctx->stream;
    const uint32_t n = (uint32_t)ctx->n;
    const bool comp = ctx->opt.precision == GC_PREC_F32_KAHAN;
    HIPCHK(launch_copy_range(ctx->B, ctx->A, ctx->n_active, ctx->n_bound, n, comp, ctx->dead, s));
    HIPCHK(launch_copy_count(ctx->n_bound, ctx->n_active, ctx->count_host, ctx->sorted_n, ctx->sc.state, s, e1));
    ctx->order_known = true;
    ctx->keys_known = order == GC_ORDER_BIN;
    std::swap(ctx->A, ctx->B);
    std::swap(ctx->soa_mem[0], ctx->soa_mem[1]);
    if (e0) ctx->ev_reorder.push_back({e0, e1, p0, p1});
    return GC_OK;
}

gc_status push(gc_ctx *ctx, double dt, int32_t steps, bool timed) {
    hipStream_t s = ctx->stream;
    PushArgs a{};
    const bool moved = ctx->pend_perm != nullptr;   // the push applies the last reorder's permutation
    a.st = moved ? ctx->B : ctx->A;
    a.src = ctx->A;
    a.perm = ctx->pend_perm;
    a.f = ctx->f;
    a.fdev = ctx->f_dev;
    a.ens = ctx->ens_dev;
    a.fx = ctx->fx;
    a.mode = ctx->fx.data ? 2 : (ctx->any_rebirth || ctx->any_wind ? 1 : 0);
    a.n_active = ctx->n_active;
    a.n_slots = (uint32_t)ctx->n;
    a.n_steps = steps;
    a.dt = dt;
    int form = ctx->opt.field_source == GC_SOURCE_MLP || ctx->opt.persistent ? 0 : push_form(ctx);
    if (form == 2 && ctx->fx.data) form = 1;      // the full equations have no quad form
    a.steps_done = ctx->steps + form;
    a.log = ctx->log;
    a.log_depth = ctx->opt.log_depth;
    a.tile = ctx->opt.tile;
    a.queue = ctx->queue;
    const bool pers = ctx->opt.persistent != 0;
    a.tail = pers && ctx->opt.field_source == GC_SOURCE_GRID ? (uint32_t)ctx->opt.tail_threshold : 0u;
    const int grid_blocks = ctx->n_cus * (1024 / ctx->opt.block_size);
    if (pers) HIPCHK(launch_fill_u32(ctx->queue, 0u, 1, s));
    // grid push: the events are attached to the push kernels' own dispatches
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        e0 = take_event(ctx);
        e1 = take_event(ctx);
    }
    if (ctx->opt.field_source == GC_SOURCE_MLP) {
        if (moved) return fail(ctx, GC_ESTATE, "the neural-field push does not apply permutations");
        if (timed) HIPCHK(hipEventRecord(e0, s));
        HIPCHK(launch_push_mlp(a, ctx->mlp.args, ctx->opt.precision, s));
        if (timed) HIPCHK(hipEventRecord(e1, s));
    } else {
        LaunchEvents ev;
        ev.start = e0;
        ev.stop = e1;
        HIPCHK(launch_push(a, ctx->opt.precision, ctx->opt.block_size, pers, form, grid_blocks, s, ev));
    }
    if (timed) ctx->ev_push.push_back({e0, e1, form});
    if (moved) {
        // the reorder's events pass to finish_reorder (and its timing list)
        hipEvent_t r0 = ctx->pend_e0, r1 = ctx->pend_e1;
        ctx->pend_perm = nullptr;
        ctx->pend_e0 = ctx->pend_e1 = nullptr;
        return finish_reorder(ctx, ctx->pend_order, r0, r1, e0, e1);
    }
    return GC_OK;
}

// Bound the host's lead: wait for the work issued kAhead calls ago, then mark
// the end of the work issued now.
gc_status keep_close(gc_ctx *ctx) {
    hipEvent_t &ev = ctx->ahead[ctx->ahead_pos];
    if (!ev) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    else HIPCHK(hipEventSynchronize(ev));
    HIPCHK(hipEventRecord(ev, ctx->stream));
    ctx->ahead_pos = (ctx->ahead_pos + 1) % kAhead;
    return GC_OK;
}

gc_status enqueue_advance(gc_ctx *ctx, double dt, int64_t n_steps, bool timed) {
    int64_t left = n_steps;
    while (left > 0) {
        const int32_t c = (int32_t)std::min<int64_t>(left, ctx->opt.chunk_steps);
        const bool tail = tail_mode(ctx) && ctx->opt.order != GC_ORDER_NONE;   // (NONE: nothing to skip)
        gc_status st = GC_OK;
        if (!tail || ctx->bound_dirty || ctx->tail_skip <= 0) {
            st = reorder(ctx, timed && ctx->opt.timing == 1, ctx->opt.order);   // (timing 2: pushes only)
            ctx->tail_skip = kTailReorderEvery - 1;
        } else {
            --ctx->tail_skip;
        }
        if (st != GC_OK) return st;
        st = push(ctx, dt, c, timed);
        if (st != GC_OK) return st;
        if (ctx->opt.tail_threshold > 0 && !ctx->capturing) {
            gc_status st2 = keep_close(ctx);
            if (st2 != GC_OK) return st2;
        }
        left -= c;
    }
    return GC_OK;
}

gc_status check_advance(gc_ctx *ctx, double dt, int64_t n_steps) {
    if (!ctx) return GC_EINVAL;
    if (!ctx->have_field) return fail(ctx, GC_ESTATE, "gc_advance before gc_load_field");
    if (!(std::isfinite(dt) && dt > 0.0)) return fail(ctx, GC_EINVAL, "dt must be finite and > 0 (got %g)", dt);
    if (n_steps < 0) return fail(ctx, GC_EINVAL, "n_steps must be >= 0");
    if (ctx->opt.field_source == GC_SOURCE_MLP && !ctx->mlp.set)
        return fail(ctx, GC_ESTATE, "field_source is the neural field but gc_mlp_set was not called");
    if (ctx->opt.field_source == GC_SOURCE_MLP && ctx->any_rebirth)
        return fail(ctx, GC_EINVAL, "rebirth is not supported with the neural field source");
    if (ctx->opt.field_source == GC_SOURCE_MLP && ctx->any_wind)
        return fail(ctx, GC_EINVAL, "wind-frame scattering is not supported with the neural field source");
    if (ctx->opt.field_source == GC_SOURCE_MLP && ctx->fx.data)
        return fail(ctx, GC_EINVAL, "the full GC terms are not supported with the neural field source");
    return GC_OK;
}

// Stage a host [nodes][nc] node array (nc = 12, or 9 padded to 12 with zeros)
// as float64 on the device and pack it into the gathers' blocked layout
// (field_layout, store type), and with rec_out also into node records
// [nr][nth][nph+1][12] of the store type; scale receives the FP16
// per-component scales.  Waits.
gc_status pack_nodes(gc_ctx *ctx, const gc_field_desc *d, const void *host, int nc, void **out, void **rec_out,
                     float scale[12], int32_t *tame) {
    hipStream_t s = ctx->stream;
    const size_t nodes = (size_t)d->nr * d->nth * d->nph;
    const size_t packed = (size_t)field_layout(d->nr, d->nth, d->nph, d->store_dtype).total;
    std::vector<double> conv;
    const double *src = static_cast<const double *>(host);
    if (d->src_dtype == GC_F32 || nc != 12) {
        conv.assign(nodes * 12, 0.0);
        for (size_t i = 0; i < nodes; ++i)
            for (int c = 0; c < nc; ++c)
                conv[i * 12 + c] = d->src_dtype == GC_F32 ? (double)static_cast<const float *>(host)[i * nc + c]
                                                          : static_cast<const double *>(host)[i * nc + c];
        src = conv.data();
    }
    *tame = 1;
    for (size_t i = 0; i < nodes * 12; ++i)
        if (!(std::fabs(src[i]) <= kTameField)) {   // NaN included
            *tame = 0;
            break;
        }
    float inv_scale[12];
    for (int c = 0; c < 12; ++c) scale[c] = inv_scale[c] = 1.0f;
    if (d->store_dtype == GC_F16) {
        double mx[12] = {0};
        for (size_t i = 0; i < nodes; ++i)
            for (int c = 0; c < 12; ++c) mx[c] = std::max(mx[c], std::fabs(src[i * 12 + c]));
        for (int c = 0; c < 12; ++c) {
            if (!(mx[c] > 0.0) || !std::isfinite(mx[c])) continue;
            const int e = (int)std::ceil(std::log2(mx[c])) - 14;   // max maps into (8192, 16384]
            scale[c] = std::ldexp(1.0f, e);
            inv_scale[c] = std::ldexp(1.0f, -e);
        }
    }
    const size_t esz = d->store_dtype == GC_F64 ? 8 : (d->store_dtype == GC_F32 ? 4 : 2);
    const size_t recs = (size_t)d->nr * d->nth * (d->nph + 1) * 12;
    void *stage = nullptr, *buf = nullptr, *rec = nullptr;
    if (dalloc(ctx, (void **)&stage, nodes * 12 * 8 + 64) != hipSuccess) return fail(ctx, GC_ENOMEM, "cannot stage field");
    if (dalloc(ctx, (void **)&buf, packed * esz) != hipSuccess ||
        (rec_out && dalloc(ctx, (void **)&rec, recs * esz) != hipSuccess)) {
        dfree(ctx, stage);
        dfree(ctx, buf);
        return fail(ctx, GC_ENOMEM, "cannot allocate field");
    }
    float *dscale = reinterpret_cast<float *>(static_cast<char *>(stage) + nodes * 12 * 8);
    hipError_t e = hipMemcpyAsync(stage, src, nodes * 12 * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dscale, inv_scale, sizeof inv_scale, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_pack_field(static_cast<const double *>(stage), buf, d->nr, d->nth, d->nph, d->store_dtype, 0,
                              dscale, s);
    if (e == hipSuccess && rec)
        e = launch_pack_field(static_cast<const double *>(stage), rec, d->nr, d->nth, d->nph, d->store_dtype, 1,
                              dscale, s);
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    dfree(ctx, stage);
    if (e != hipSuccess) {
        dfree(ctx, buf);
        dfree(ctx, rec);
        return fail(ctx, GC_EDEVICE, "field packing: %s", hipGetErrorString(e));
    }
    *out = buf;
    if (rec_out) *rec_out = rec;
    return GC_OK;
}

}  // namespace

extern "C" {

void gc_default_options(gc_options *o) {
    std::memset(o, 0, sizeof *o);
    o->precision = GC_PREC_F64;
    o->order = GC_ORDER_BIN;
    o->chunk_steps = 64;
    o->bin_coarsen = 0;
    o->block_size = 64;
    o->persistent = 0;
    o->tile = 1024;
    o->log_depth = 0;
    o->timing = 0;
    o->field_source = GC_SOURCE_GRID;
    o->tail_threshold = 131072;
}

gc_status gc_create(gc_ctx **out, const gc_options *opt) {
    if (!out) return GC_EINVAL;
    *out = nullptr;
    gc_options o;
    if (opt) o = *opt;
    else gc_default_options(&o);
    gc_ctx *ctx = new gc_ctx();
    ctx->opt = o;
    gc_status st = check_options(ctx, &o);
    if (st != GC_OK) {
        *out = ctx;   // the caller can read the message, then destroy
        return st;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || o.device < 0 || o.device >= ndev) {
        *out = ctx;
        return fail(ctx, GC_EDEVICE, "no HIP device %d (count %d)", o.device, ndev);
    }
    *out = ctx;
    HIPCHK(hipSetDevice(o.device));
    scratch_init(o.device);
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, o.device));
    ctx->n_cus = prop.multiProcessorCount;
    ctx->stream = static_cast<hipStream_t>(o.hip_stream);
    ctx->ens_host.assign(kMaxEnsembles, EnsDev{});
    ctx->ens_set.assign(kMaxEnsembles, 0);
    HIPCHK(dalloc(ctx, (void **)&ctx->ens_dev, sizeof(EnsDev) * kMaxEnsembles));
    HIPCHK(dalloc(ctx, (void **)&ctx->f_dev, sizeof(FieldDev)));
    void *small = nullptr;
    HIPCHK(dalloc(ctx, (void **)&small, 256));
    ctx->n_active = static_cast<uint32_t *>(small);
    ctx->queue = ctx->n_active + 1;
    ctx->n_bound = ctx->n_active + 2;
    ctx->sorted_n = ctx->n_active + 3;
    ctx->steps = reinterpret_cast<unsigned long long *>(static_cast<char *>(small) + 64);
    ctx->dead = reinterpret_cast<unsigned long long *>(static_cast<char *>(small) + 128);
    HIPCHK(launch_fill_u32(ctx->n_active, 0u, 4, ctx->stream));
    HIPCHK(launch_fill_u64(ctx->steps, 0ull, kPushForms, ctx->stream));
    HIPCHK(launch_fill_u64(ctx->dead, 0ull, 8, ctx->stream));
    void *pinned = nullptr;
    HIPCHK(hipHostMalloc(&pinned, 64, hipHostMallocCoherent));
    ctx->count_host = static_cast<volatile uint32_t *>(pinned);
    *ctx->count_host = 0xFFFFFFFFu;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return GC_OK;
}

void gc_destroy(gc_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    for (auto &p : ctx->ev_push) {
        (void)hipEventDestroy(p.e0);
        (void)hipEventDestroy(p.e1);
    }
    for (auto &p : ctx->ev_reorder) {
        (void)hipEventDestroy(p.e0);
        (void)hipEventDestroy(p.e1);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : {ctx->pend_e0, ctx->pend_e1})
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->ahead)
        if (e) (void)hipEventDestroy(e);
    for (int i = 0; i < 2; ++i)
        if (ctx->soa_mem[i]) dfree(ctx, ctx->soa_mem[i]);
    if (ctx->scratch_mem) dfree(ctx, ctx->scratch_mem);
    if (ctx->log) dfree(ctx, ctx->log);
    if (ctx->field_buf) dfree(ctx, ctx->field_buf);
    if (ctx->field_rec_buf) dfree(ctx, ctx->field_rec_buf);
    if (ctx->extra_buf) dfree(ctx, ctx->extra_buf);
    if (ctx->mlp.mem) dfree(ctx, ctx->mlp.mem);
    if (ctx->mlp.ws) dfree(ctx, ctx->mlp.ws);
    if (ctx->ens_dev) dfree(ctx, ctx->ens_dev);
    if (ctx->f_dev) dfree(ctx, ctx->f_dev);
    if (ctx->n_active) dfree(ctx, ctx->n_active);
    if (ctx->count_host) (void)hipHostFree(const_cast<uint32_t *>(ctx->count_host));
    delete ctx;
}

const char *gc_last_error(const gc_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gc_status gc_set_options(gc_ctx *ctx, const gc_options *opt) {
    if (!ctx || !opt) return GC_EINVAL;
    gc_options o = *opt;
    o.dev_alloc = ctx->opt.dev_alloc;      // the allocator is fixed at creation
    o.dev_free = ctx->opt.dev_free;
    o.alloc_user = ctx->opt.alloc_user;
    if (o.log_depth != ctx->opt.log_depth) return fail(ctx, GC_EINVAL, "log_depth cannot change after creation");
    if (o.device != ctx->opt.device) return fail(ctx, GC_EINVAL, "device cannot change after creation");
    gc_status st = check_options(ctx, &o);
    if (st != GC_OK) return st;
    const bool was_kahan = ctx->opt.precision == GC_PREC_F32_KAHAN, is_kahan = o.precision == GC_PREC_F32_KAHAN;
    if (o.order != ctx->opt.order || was_kahan != is_kahan) ctx->bound_dirty = true;
    ctx->opt = o;
    ctx->stream = static_cast<hipStream_t>(o.hip_stream);
    if (was_kahan != is_kahan && ctx->n > 0) {
        // compensation terms only follow the particles in the Kahan form: restart them at zero
        double *comp[5] = {ctx->A.cr, ctx->A.cth, ctx->A.cph, ctx->A.cu, ctx->A.ct};
        for (double *c : comp)
            HIPCHK(launch_fill_u64(reinterpret_cast<unsigned long long *>(c), 0ull, ctx->n, ctx->stream));
    }
    return GC_OK;
}

gc_status gc_get_options(const gc_ctx *ctx, gc_options *opt) {
    if (!ctx || !opt) return GC_EINVAL;
    *opt = ctx->opt;
    return GC_OK;
}

gc_status gc_load_field(gc_ctx *ctx, const gc_field_desc *d) {
    if (!ctx || !d) return GC_EINVAL;
    if (d->nr < 2 || d->nth < 2 || d->nph < 2)
        return fail(ctx, GC_EINVAL, "grid needs at least 2 nodes per axis (%d, %d, %d)", d->nr, d->nth, d->nph);
    if (!(d->r_min > 0.0) || !(d->r_max > d->r_min)) return fail(ctx, GC_EINVAL, "need 0 < r_min < r_max");
    if (!d->data) return fail(ctx, GC_EINVAL, "data is NULL");
    if (d->src_dtype != GC_F64 && d->src_dtype != GC_F32) return fail(ctx, GC_EINVAL, "src_dtype must be F64 or F32");
    if (d->store_dtype < GC_F64 || d->store_dtype > GC_F16) return fail(ctx, GC_EINVAL, "unknown store_dtype");
    const FieldLayout lay = field_layout(d->nr, d->nth, d->nph, d->store_dtype);
    const uint64_t esz = d->store_dtype == GC_F64 ? 8 : (d->store_dtype == GC_F32 ? 4 : 2);
    if ((uint64_t)d->nr * d->nth * d->nph > 0x7FFFFFFFull || lay.total * esz > 0xFFFFFFFFull)
        return fail(ctx, GC_EINVAL, "packed field larger than 4 GiB (%llu bytes; 32-bit load offsets)",
                    (unsigned long long)(lay.total * esz));
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    float scale[12], xscale[12];
    int32_t tame = 0, xtame = 0;
    void *buf = nullptr, *rbuf = nullptr, *xbuf = nullptr;
    // node records for the four-lanes-per-particle form (FP32 and FP64 stores)
    gc_status st = pack_nodes(ctx, d, d->data, 12, &buf, d->store_dtype == GC_F16 ? nullptr : &rbuf, scale, &tame);
    if (st != GC_OK) return st;
    if (d->extra) {
        st = pack_nodes(ctx, d, d->extra, 9, &xbuf, nullptr, xscale, &xtame);
        if (st != GC_OK) {
            dfree(ctx, buf);
            dfree(ctx, rbuf);
            return st;
        }
    }
    if (ctx->field_buf) dfree(ctx, ctx->field_buf);
    if (ctx->field_rec_buf) dfree(ctx, ctx->field_rec_buf);
    if (ctx->extra_buf) dfree(ctx, ctx->extra_buf);
    ctx->field_buf = buf;
    ctx->field_rec_buf = rbuf;
    ctx->extra_buf = xbuf;
    FieldDev &f = ctx->f;
    f.data = buf;
    f.nr = d->nr;
    f.nth = d->nth;
    f.nph = d->nph;
    f.dtype = d->store_dtype;
    f.r_min = d->r_min;
    const double pi = 3.14159265358979323846;
    f.inv_dr = (double)(d->nr - 1) / (d->r_max - d->r_min);
    f.inv_dth = (double)d->nth / pi;
    f.inv_dph = (double)d->nph / (2.0 * pi);
    f.inv_nph = 1.0 / (double)d->nph;
    f.th_lo = 0.5 * pi / d->nth;
    f.th_hi = pi - 0.5 * pi / d->nth;
    for (int c = 0; c < 12; ++c) f.scale[c] = scale[c];
    f.cs = lay.cs;
    f.ks = lay.ks;
    f.js = lay.js;
    f.rec = rbuf;
    f.tame = tame;
    ctx->fx = f;                      // same geometry, the extra node array (or none)
    ctx->fx.data = xbuf;
    ctx->fx.rec = nullptr;
    ctx->fx.tame = xtame;
    if (xbuf)
        for (int c = 0; c < 12; ++c) ctx->fx.scale[c] = xscale[c];
    HIPCHK(hipMemcpyAsync(ctx->f_dev, &ctx->f, sizeof(FieldDev), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    ctx->have_field = true;
    if (ctx->gexec) {
        (void)hipGraphExecDestroy(ctx->gexec);
        ctx->gexec = nullptr;
    }
    return GC_OK;
}

gc_status gc_inject(gc_ctx *ctx, const gc_inject_desc *d) {
    if (!ctx || !d) return GC_EINVAL;
    if (!ctx->have_field) return fail(ctx, GC_ESTATE, "gc_inject before gc_load_field");
    if (d->ensemble >= (uint32_t)kMaxEnsembles) return fail(ctx, GC_EINVAL, "ensemble index >= %d", kMaxEnsembles);
    if (!(d->m > 0.0) || d->q == 0.0 || !std::isfinite(d->q)) return fail(ctx, GC_EINVAL, "need m > 0 and q != 0");
    if (!(d->ekin > 0.0) || !std::isfinite(d->ekin)) return fail(ctx, GC_EINVAL, "need ekin > 0");
    if (!(d->r_in < d->r_out)) return fail(ctx, GC_EINVAL, "need r_in < r_out");
    if (!(d->mu_lo >= -1.0 && d->mu_lo <= 1.0 && d->mu_hi >= -1.0 && d->mu_hi <= 1.0))
        return fail(ctx, GC_EINVAL, "mu_lo and mu_hi must be in [-1, 1]");
    if (d->scatter_law != 0 && d->scatter_law != 1) return fail(ctx, GC_EINVAL, "scatter_law must be 0 or 1");
    if (d->rebirth_steps > (int64_t)kMaxRebirthSteps)
        return fail(ctx, GC_EINVAL, "rebirth_steps must be <= %lld", (long long)kMaxRebirthSteps);
    if (!(d->v_wind >= 0.0 && d->v_wind < 0.1 * 299792458.0))
        return fail(ctx, GC_EINVAL, "v_wind must be in [0, 0.1 c)");
    if (d->n == 0) return GC_OK;
    if ((uint64_t)d->first_id + d->n > 0x100000000ull) return fail(ctx, GC_EINVAL, "ids exceed 32 bits");
    HIPCHK(hipSetDevice(ctx->opt.device));
    gc_status st = reserve(ctx, ctx->n + d->n);
    if (st != GC_OK) return st;
    EnsDev e{};
    e.qm = d->q / d->m;
    e.iqm = d->m / d->q;
    e.m = d->m;
    e.lambda = d->lambda_par;
    e.r_in = d->r_in;
    e.r_out = d->r_out;
    e.seed = d->seed;
    e.max_steps = d->max_steps;
    e.ensemble = d->ensemble;
    e.drift_free = d->drift_free ? 1 : 0;
    e.scatter_law = d->scatter_law;
    e.ekin = d->ekin;
    e.r0 = d->r0;
    e.lat0 = d->lat0;
    e.lon0 = d->lon0;
    e.dlon = d->dlon;
    e.dr0 = d->dr0;
    e.dlat = d->dlat;
    e.mu_lo = d->mu_lo;
    e.mu_hi = d->mu_hi;
    e.rebirth_steps = d->rebirth_steps;
    e.v_wind = d->v_wind;
    ctx->ens_host[d->ensemble] = e;
    ctx->ens_set[d->ensemble] = 1;
    ctx->any_rebirth = false;
    ctx->any_wind = false;
    for (int i = 0; i < kMaxEnsembles; ++i) {
        if (!ctx->ens_set[i]) continue;
        if (ctx->ens_host[i].rebirth_steps > 0) ctx->any_rebirth = true;
        if (ctx->ens_host[i].v_wind > 0.0) ctx->any_wind = true;
    }
    HIPCHK(hipMemcpyAsync(ctx->ens_dev + d->ensemble, &ctx->ens_host[d->ensemble], sizeof(EnsDev),
                          hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(launch_inject(ctx->A, ctx->f, e, (uint32_t)ctx->n, (uint32_t)d->n, d->first_id, d->ensemble,
                         ctx->stream));
    ctx->n += d->n;
    ctx->bound_dirty = true;
    ctx->order_known = ctx->keys_known = false;
    if (ctx->count_host) *ctx->count_host = 0xFFFFFFFFu;
    return GC_OK;
}

gc_status gc_advance(gc_ctx *ctx, double dt, int64_t n_steps) {
    gc_status st = check_advance(ctx, dt, n_steps);
    if (st != GC_OK) return st;
    if (ctx->n == 0 || n_steps == 0) return GC_OK;
    HIPCHK(hipSetDevice(ctx->opt.device));
    return enqueue_advance(ctx, dt, n_steps, ctx->opt.timing != 0);
}

gc_status gc_advance_graph(gc_ctx *ctx, double dt, int64_t n_steps) {
    gc_status st = check_advance(ctx, dt, n_steps);
    if (st != GC_OK) return st;
    if (ctx->n == 0 || n_steps == 0) return GC_OK;
    if (!ctx->stream) return fail(ctx, GC_EINVAL, "graph capture needs a non-null stream");
    HIPCHK(hipSetDevice(ctx->opt.device));
    // The tail: once the live count read back is below tail_threshold, a replay
    // would mostly pay for its fixed launches (a reorder every chunk); the chunks
    // then run eagerly with the tail policy (bitwise the same results).
    if (tail_mode(ctx) && ctx->opt.order != GC_ORDER_NONE) return enqueue_advance(ctx, dt, n_steps, ctx->opt.timing != 0);
    // reset the live prefix now, never inside a graph: captured, the reset would
    // make every replay sort and copy the stopped particles again
    if (ctx->bound_dirty && ctx->opt.order != GC_ORDER_NONE) {
        HIPCHK(launch_reset_bound(ctx->n_bound, (uint32_t)ctx->n, ctx->dead, ctx->stream));
        ctx->bound_dirty = false;
    }
    const bool same = ctx->gexec && ctx->gkey.dt == dt && ctx->gkey.n_steps == n_steps && ctx->gkey.n == ctx->n &&
                      ctx->gkey.state == ctx->soa_mem[0] &&
                      std::memcmp(&ctx->gkey.opt, &ctx->opt, sizeof(gc_options)) == 0;
    if (!same) {
        if (ctx->gexec) {
            (void)hipGraphExecDestroy(ctx->gexec);
            ctx->gexec = nullptr;
        }
        // the number of reorders must be even so that the state ends in the buffer it started in
        const int64_t chunks = (n_steps + ctx->opt.chunk_steps - 1) / ctx->opt.chunk_steps;
        if (ctx->opt.order != GC_ORDER_NONE && (chunks & 1))
            return fail(ctx, GC_EINVAL, "graph mode needs an even number of chunks (n_steps / chunk_steps)");
        HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        ctx->capturing = true;
        st = enqueue_advance(ctx, dt, n_steps, false);
        ctx->capturing = false;
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(ctx->stream, &g);
        if (st != GC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        HIPCHK(ce);
        hipGraphExec_t ex = nullptr;
        hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(ie);
        ctx->gexec = ex;
        ctx->gkey.dt = dt;
        ctx->gkey.n_steps = n_steps;
        ctx->gkey.n = ctx->n;
        ctx->gkey.state = ctx->soa_mem[0];
        ctx->gkey.opt = ctx->opt;
    }
    HIPCHK(hipGraphLaunch(ctx->gexec, ctx->stream));
    if (ctx->opt.tail_threshold > 0) return keep_close(ctx);   // keeps the count read back recent
    return GC_OK;
}

int64_t gc_moments_size(const gc_moment_spec *s) {
    if (!s) return -1;
    return 8 + 3 * (int64_t)s->n_rbins + s->n_mubins + (int64_t)s->n_agebins * s->n_ebins;
}

gc_status gc_moments(gc_ctx *ctx, const gc_moment_spec *s, int64_t *out) {
    if (!ctx || !s) return GC_EINVAL;
    if (!out) return fail(ctx, GC_EINVAL, "out is NULL");
    if (!ctx->have_field) return fail(ctx, GC_ESTATE, "gc_moments before gc_load_field");
    if (s->n_rbins < 0 || s->n_mubins < 0 || s->n_agebins < 0 || s->n_ebins < 0)
        return fail(ctx, GC_EINVAL, "negative bin count");
    if (s->n_rbins > 0 && !(s->r_hi > s->r_lo)) return fail(ctx, GC_EINVAL, "empty radial range");
    if (s->n_agebins > 0 && !(s->age_max > 0.0)) return fail(ctx, GC_EINVAL, "age_max must be > 0");
    if (s->n_ebins > 0 && !(s->e_hi > s->e_lo)) return fail(ctx, GC_EINVAL, "empty energy range");
    if (!(s->e_unit > 0.0) || !(s->len_unit > 0.0)) return fail(ctx, GC_EINVAL, "e_unit and len_unit must be > 0");
    const int64_t total = gc_moments_size(s);
    if (total > kMaxMoments) return fail(ctx, GC_EINVAL, "too many moment outputs (%lld > %d)", (long long)total, kMaxMoments);
    HIPCHK(hipSetDevice(ctx->opt.device));
    MomDev m{};
    m.n_rbins = s->n_rbins;
    m.n_mubins = s->n_mubins;
    m.n_agebins = s->n_agebins;
    m.n_ebins = s->n_ebins;
    m.min_collisions = s->min_collisions;
    m.total = (int32_t)total;
    m.r_lo = s->r_lo;
    m.r_hi = s->r_hi;
    m.sel_r_lo = s->sel_r_lo;
    m.sel_r_hi = s->sel_r_hi;
    m.age_lo = s->age_lo;
    m.age_hi = s->age_hi;
    m.age_max = s->age_max;
    m.e_lo = s->e_lo;
    m.e_hi = s->e_hi;
    m.e_unit = s->e_unit;
    m.len_unit = s->len_unit;
    m.min_birth = s->min_birth;
    m.accumulate = s->accumulate != 0;
    // after a reorder only the live prefix is read; the sums over the slots
    // past it are kept on the device by the reorders
    HIPCHK(launch_moments(ctx->A, ctx->f, ctx->ens_dev, (uint32_t)ctx->n, m,
                          reinterpret_cast<unsigned long long *>(out), ctx->bound_dirty ? nullptr : ctx->n_bound,
                          ctx->bound_dirty ? nullptr : ctx->dead, ctx->stream));
    return GC_OK;
}

gc_status gc_count(const gc_ctx *ctx, uint64_t *n) {
    if (!ctx || !n) return GC_EINVAL;
    *n = ctx->n;
    return GC_OK;
}

gc_status gc_get_state(gc_ctx *ctx, const gc_state_view *dst) {
    if (!ctx || !dst) return GC_EINVAL;
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(launch_state_out(ctx->A, *dst, (uint32_t)ctx->n, ctx->stream));
    return GC_OK;
}

gc_status gc_set_state(gc_ctx *ctx, const gc_state_view *src, uint64_t n) {
    if (!ctx || !src) return GC_EINVAL;
    if (!ctx->have_field) return fail(ctx, GC_ESTATE, "gc_set_state before gc_load_field");
    const void *ptrs[] = {src->r, src->th, src->ph, src->u, src->mu, src->fr, src->fth, src->fph, src->fu,
                          src->dtp, src->s, src->ell, src->t, src->cr, src->cth, src->cph, src->cu, src->ct,
                          src->k, src->flags, src->status, src->step, src->id, src->ens, src->birth};
    for (const void *p : ptrs)
        if (!p) return fail(ctx, GC_EINVAL, "every member of the state view must be set");
    HIPCHK(hipSetDevice(ctx->opt.device));
    gc_status st = reserve(ctx, n);
    if (st != GC_OK) return st;
    HIPCHK(launch_state_in(ctx->A, *src, (uint32_t)n, ctx->stream));
    // a fresh state: an earlier failed sort pass no longer taints it, and a
    // reorder cut short by a failed advance leaves no counts, tickets or
    // look-back tags behind (the reset also moves the tags to a new epoch)
    if (ctx->sc.state) {
        HIPCHK(launch_fill_u32(ctx->sc.state + kStError, 0u, 1, ctx->stream));
        HIPCHK(launch_copy_count(ctx->n_bound, ctx->n_active, nullptr, nullptr, ctx->sc.state, ctx->stream));
    }
    if (ctx->pend_perm) {
        ctx->pend_perm = nullptr;
        for (hipEvent_t e : {ctx->pend_e0, ctx->pend_e1})
            if (e) ctx->ev_pool.push_back(e);
        ctx->pend_e0 = ctx->pend_e1 = nullptr;
    }
    ctx->n = n;
    ctx->bound_dirty = true;
    ctx->order_known = ctx->keys_known = false;
    if (ctx->count_host) *ctx->count_host = 0xFFFFFFFFu;
    if (ctx->gexec) {
        (void)hipGraphExecDestroy(ctx->gexec);
        ctx->gexec = nullptr;
    }
    return GC_OK;
}

gc_status gc_get_log(gc_ctx *ctx, uint32_t *dst) {
    if (!ctx || !dst) return GC_EINVAL;
    if (ctx->opt.log_depth <= 0) return fail(ctx, GC_ESTATE, "collision log is off (log_depth = 0)");
    if (ctx->n == 0) return GC_OK;
    HIPCHK(hipMemcpyAsync(dst, ctx->log, ctx->n * ctx->opt.log_depth * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                          ctx->stream));
    return GC_OK;
}

gc_status gc_get_order(gc_ctx *ctx, uint32_t *slot_gid, uint32_t *slot_key, uint32_t *n_live) {
    if (!ctx) return GC_EINVAL;
    if (!slot_gid && !slot_key && !n_live) return fail(ctx, GC_EINVAL, "no output given");
    if (!ctx->order_known) return fail(ctx, GC_ESTATE, "no reorder since the particle set last changed");
    if (slot_key && !ctx->keys_known) return fail(ctx, GC_ESTATE, "the last reorder was not a cell binning");
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    const uint32_t n = (uint32_t)ctx->n;
    if (slot_gid && n) HIPCHK(hipMemcpyAsync(slot_gid, ctx->A.gid, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    if (slot_key) HIPCHK(launch_keys_out(ctx->sc.sorted_keys, ctx->sorted_n, ctx->sorted_dead, n, slot_key, s));
    if (n_live) HIPCHK(hipMemcpyAsync(n_live, ctx->n_active, 4, hipMemcpyDeviceToDevice, s));
    return GC_OK;
}

gc_status gc_get_counters(gc_ctx *ctx, gc_counters *out) {
    if (!ctx || !out) return GC_EINVAL;
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::memset(out, 0, sizeof *out);
    for (auto &p : ctx->ev_push) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, p.e0, p.e1));
        out->push_ms += ms;
        out->n_push += 1;
        out->form_ms[p.form] += ms;
        out->form_launches[p.form] += 1;
    }
    for (auto &p : ctx->ev_reorder) {
        float ms = 0, pm = 0;
        HIPCHK(hipEventElapsedTime(&ms, p.e0, p.e1));
        if (p.p0) HIPCHK(hipEventElapsedTime(&pm, p.p0, p.p1));
        out->reorder_ms += ms - pm;
        out->n_reorder += 1;
    }
    unsigned long long steps[kPushForms] = {0, 0, 0};
    HIPCHK(hipMemcpy(steps, ctx->steps, sizeof steps, hipMemcpyDeviceToHost));
    uint32_t sort_error = 0;
    if (ctx->sc.state) HIPCHK(hipMemcpy(&sort_error, ctx->sc.state + kStError, 4, hipMemcpyDeviceToHost));
    if (sort_error) return fail(ctx, GC_EDEVICE, "a radix-sort pass gave up waiting for a tile: the particle order is invalid");
    for (int f = 0; f < kPushForms; ++f) {
        out->form_steps[f] = steps[f];
        out->particle_steps += steps[f];
    }
    return GC_OK;
}

gc_status gc_reset_counters(gc_ctx *ctx) {
    if (!ctx) return GC_EINVAL;
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (auto &p : ctx->ev_push) {
        ctx->ev_pool.push_back(p.e0);
        ctx->ev_pool.push_back(p.e1);
    }
    ctx->ev_push.clear();
    for (auto &p : ctx->ev_reorder) {   // (p0, p1 belong to ev_push)
        ctx->ev_pool.push_back(p.e0);
        ctx->ev_pool.push_back(p.e1);
    }
    ctx->ev_reorder.clear();
    HIPCHK(launch_fill_u64(ctx->steps, 0ull, kPushForms, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return GC_OK;
}

}  // extern "C"

namespace {

// Device copy of the whole state in global order, for the autotuner.
struct Snapshot {
    gc_ctx *ctx = nullptr;
    void *mem = nullptr;
    gc_state_view v{};
    uint64_t n = 0;
    ~Snapshot() {
        if (mem) {
            (void)hipStreamSynchronize(ctx->stream);   // queued copies may still read it
            dfree(ctx, mem);
        }
    }
};

gc_status take_snapshot(gc_ctx *ctx, Snapshot &sn) {
    sn.ctx = ctx;
    sn.n = ctx->n;
    const size_t bytes = (size_t)sn.n * (kNumDoubleArrays * 8 + 7 * 4) + 64;
    if (dalloc(ctx, (void **)&sn.mem, bytes) != hipSuccess) return fail(ctx, GC_ENOMEM, "cannot allocate tuning snapshot");
    double *d = static_cast<double *>(sn.mem);
    double **dp[kNumDoubleArrays] = {&sn.v.r, &sn.v.th, &sn.v.ph, &sn.v.u, &sn.v.mu, &sn.v.fr, &sn.v.fth, &sn.v.fph,
                                     &sn.v.fu, &sn.v.dtp, &sn.v.s, &sn.v.ell, &sn.v.t, &sn.v.cr, &sn.v.cth, &sn.v.cph,
                                     &sn.v.cu, &sn.v.ct};
    for (int i = 0; i < kNumDoubleArrays; ++i) *dp[i] = d + (size_t)i * sn.n;
    uint32_t *u = reinterpret_cast<uint32_t *>(d + (size_t)kNumDoubleArrays * sn.n);
    uint32_t **up[7] = {&sn.v.k, &sn.v.flags, &sn.v.status, &sn.v.step, &sn.v.id, &sn.v.ens, &sn.v.birth};
    for (int i = 0; i < 7; ++i) *up[i] = u + (size_t)i * sn.n;
    return gc_get_state(ctx, &sn.v);
}

// Rate of one candidate: restore, advance probe_steps, time with events.
gc_status time_candidate(gc_ctx *ctx, const Snapshot &sn, const gc_options &o, double dt, int64_t steps,
                         double *rate) {
    gc_status st = gc_set_options(ctx, &o);
    if (st != GC_OK) return st;
    st = gc_set_state(ctx, &sn.v, sn.n);
    if (st != GC_OK) return st;
    hipStream_t s = ctx->stream;
    HIPCHK(launch_fill_u64(ctx->steps, 0ull, kPushForms, s));
    hipEvent_t e0 = take_event(ctx), e1 = take_event(ctx);
    HIPCHK(hipEventRecord(e0, s));
    st = enqueue_advance(ctx, dt, steps, false);
    if (st != GC_OK) return st;
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    ctx->ev_pool.push_back(e0);
    ctx->ev_pool.push_back(e1);
    unsigned long long done[kPushForms] = {0, 0, 0};
    HIPCHK(hipMemcpy(done, ctx->steps, sizeof done, hipMemcpyDeviceToHost));
    const double total = (double)done[0] + (double)done[1] + (double)done[2];
    *rate = ms > 0 ? total / (ms * 1e-3) : 0.0;
    return GC_OK;
}

}  // namespace

gc_status gc_autotune(gc_ctx *ctx, const gc_tune_space *sp, gc_tune_result *out) {
    if (!ctx || !sp || !out) return GC_EINVAL;
    if (!ctx->have_field) return fail(ctx, GC_ESTATE, "gc_autotune before gc_load_field");
    if (ctx->n == 0) return fail(ctx, GC_ESTATE, "gc_autotune needs particles");
    if (sp->probe_steps < 1) return fail(ctx, GC_EINVAL, "probe_steps must be >= 1");
    if (!(std::isfinite(sp->dt) && sp->dt > 0.0)) return fail(ctx, GC_EINVAL, "dt must be finite and > 0");
    if (sp->n_block < 0 || sp->n_block > 3 || sp->n_coarsen < 0 || sp->n_coarsen > 4 || sp->n_chunk < 0 ||
        sp->n_chunk > 6 || sp->n_tile < 0 || sp->n_tile > 4)
        return fail(ctx, GC_EINVAL, "too many candidates");
    HIPCHK(hipSetDevice(ctx->opt.device));
    Snapshot sn;
    gc_status st = take_snapshot(ctx, sn);
    if (st != GC_OK) return st;
    const gc_options entry = ctx->opt;
    unsigned long long counter_saved[kPushForms] = {0, 0, 0};
    HIPCHK(hipMemcpy(counter_saved, ctx->steps, sizeof counter_saved, hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof *out);
    gc_options best = entry;
    best.timing = 0;
    double best_rate = 0;
    st = time_candidate(ctx, sn, best, sp->dt, sp->probe_steps, &best_rate);
    if (st != GC_OK) return st;
    out->default_rate = best_rate;
    out->n_tried = 1;
    auto consider = [&](gc_options cand) -> gc_status {
        double r = 0;
        gc_status s2 = time_candidate(ctx, sn, cand, sp->dt, sp->probe_steps, &r);
        if (s2 != GC_OK) return s2;
        out->n_tried += 1;
        if (r > best_rate) {
            best_rate = r;
            best = cand;
        }
        return GC_OK;
    };
    for (int i = 0; i < sp->n_block; ++i) {
        gc_options c = best;
        c.block_size = sp->block[i];
        if (c.persistent) c.tile = (c.tile + c.block_size - 1) / c.block_size * c.block_size;
        if (c.block_size != best.block_size && (st = consider(c)) != GC_OK) return st;
    }
    for (int i = 0; i < sp->n_coarsen; ++i) {
        gc_options c = best;
        c.bin_coarsen = sp->coarsen[i];
        if (c.bin_coarsen != best.bin_coarsen && (st = consider(c)) != GC_OK) return st;
    }
    for (int i = 0; i < sp->n_chunk; ++i) {
        gc_options c = best;
        c.chunk_steps = sp->chunk[i];
        if (c.chunk_steps != best.chunk_steps && (st = consider(c)) != GC_OK) return st;
    }
    for (int i = 0; i < sp->n_tile; ++i) {
        gc_options c = best;
        c.persistent = 1;
        c.tile = (sp->tile[i] + c.block_size - 1) / c.block_size * c.block_size;
        if ((st = consider(c)) != GC_OK) return st;
    }
    // apply the winner, restore the particles and the step counter
    best.timing = entry.timing;
    best.hip_stream = entry.hip_stream;
    st = gc_set_options(ctx, &best);
    if (st != GC_OK) return st;
    st = gc_set_state(ctx, &sn.v, sn.n);
    if (st != GC_OK) return st;
    HIPCHK(hipMemcpyAsync(ctx->steps, counter_saved, sizeof counter_saved, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    out->best = best;
    out->best_rate = best_rate;
    return GC_OK;
}

extern "C" {

gc_status gc_gather_probe(gc_ctx *ctx, double dt, int32_t n_steps, double *sink) {
    if (!ctx) return GC_EINVAL;
    if (!ctx->have_field) return fail(ctx, GC_ESTATE, "gc_gather_probe before gc_load_field");
    if (!(std::isfinite(dt) && dt > 0.0) || n_steps < 0) return fail(ctx, GC_EINVAL, "need dt > 0 and n_steps >= 0");
    if (ctx->n == 0 || n_steps == 0) return GC_OK;
    if (!sink) return fail(ctx, GC_EINVAL, "sink is NULL");
    HIPCHK(hipSetDevice(ctx->opt.device));
    PushArgs a{};
    a.st = ctx->A;
    a.src = ctx->A;
    a.f = ctx->f;
    a.ens = ctx->ens_dev;
    a.n_active = ctx->bound_dirty ? nullptr : ctx->n_active;
    a.n_slots = (uint32_t)ctx->n;
    a.n_steps = n_steps;
    a.dt = dt;
    a.steps_done = ctx->steps;
    if (!a.n_active) {
        // no reorder since the last change of the particle set: visit all slots
        HIPCHK(launch_set_count(ctx->queue, (uint32_t)ctx->n, ctx->stream));
        a.n_active = ctx->queue;
    }
    HIPCHK(launch_gather_probe(a, sink, ctx->opt.block_size, ctx->stream));
    return GC_OK;
}

gc_status gc_copy_probe(gc_ctx *ctx, void *dst, const void *src, uint64_t n_bytes) {
    if (!ctx || !dst || !src) return GC_EINVAL;
    if (n_bytes % 16) return fail(ctx, GC_EINVAL, "n_bytes must be a multiple of 16");
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(launch_copy_probe(dst, src, n_bytes, ctx->stream));
    return GC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Neural field
// ---------------------------------------------------------------------------
namespace {

constexpr int kUserParams = GC_MLP_PARAMS;             // W | c | W_o[6][128] | c_o[6]
constexpr int kUserOffWo = kMlpOffWo, kUserOffCo = kMlpOffWo + kMlpOut * kMlpWidth;
static_assert(kUserOffCo + kMlpOut == kUserParams, "GC_MLP_PARAMS does not match the network shape");
constexpr int kTrainGroups = 128;                     // most row groups of the split-K weight gradients
constexpr int kRowsPerGroup = 128;
constexpr int kLossBlocks = 512;

void to_device_layout(const float *u, std::vector<float> &d) {
    d.assign(kMlpParams, 0.0f);
    if (!u) return;
    std::copy(u, u + kUserOffWo, d.begin());          // W and c share the layout
    std::copy(u + kUserOffWo, u + kUserOffCo, d.begin() + kMlpOffWo);
    std::copy(u + kUserOffCo, u + kUserParams, d.begin() + kMlpOffCo);
}

void to_user_layout(const std::vector<float> &d, float *u) {
    std::copy(d.begin(), d.begin() + kUserOffWo, u);
    std::copy(d.begin() + kMlpOffWo, d.begin() + kMlpOffWo + kMlpOut * kMlpWidth, u + kUserOffWo);
    std::copy(d.begin() + kMlpOffCo, d.begin() + kMlpOffCo + kMlpOut, u + kUserOffCo);
}

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Partials of the training step for R rows: the split-K weight gradients
// (row groups, at most kTrainGroups), and the column sums of the output layer
// (one block per kColRows rows, plus the summed block).
constexpr size_t ws_part_floats(size_t R, size_t wgrad_groups) {
    return std::max<size_t>(wgrad_groups * kMlpWidth * kMlpWidth,
                            (size_t)(mlp_col_groups((int)std::min<size_t>(R, 1u << 30)) + 1) *
                                (kMlpOut * kMlpWidth + kMlpOut));
}

// Bytes of the training workspace for R rows; with base, also carve it.
constexpr size_t ws_bytes(size_t R, size_t part) {
    return align256(7 * R * kMlpWidth * 2) + align256(R * kMlpWidth * 2) + align256(6 * R * kMlpWidth * 4) +
           2 * align256(R * kMlpOut * 4) + align256(R * kMlpWidth * 4) + align256(part * 4) +
           align256(kLossBlocks * 8);
}

void carve_ws(char *c, size_t R, size_t part, TrainWs &w) {
    w.H = reinterpret_cast<__bf16 *>(c); c += align256(7 * R * kMlpWidth * 2);
    w.dZ = reinterpret_cast<__bf16 *>(c); c += align256(R * kMlpWidth * 2);
    w.Z = reinterpret_cast<float *>(c); c += align256(6 * R * kMlpWidth * 4);
    w.Y = reinterpret_cast<float *>(c); c += align256(R * kMlpOut * 4);
    w.dY = reinterpret_cast<float *>(c); c += align256(R * kMlpOut * 4);
    w.dH = reinterpret_cast<float *>(c); c += align256(R * kMlpWidth * 4);
    w.part = reinterpret_cast<float *>(c); c += align256(part * 4);
    w.loss_part = reinterpret_cast<double *>(c);
}

gc_status mlp_workspace(gc_ctx *ctx, int64_t rows) {
    MlpState &m = ctx->mlp;
    if (rows <= m.ws_rows) return GC_OK;
    const int64_t cap = std::max<int64_t>(rows, 2 * m.ws_rows);
    const size_t R = (size_t)cap;
    const size_t part = ws_part_floats(R, kTrainGroups);
    void *mem = nullptr;
    if (dalloc(ctx, (void **)&mem, ws_bytes(R, part)) != hipSuccess)
        return fail(ctx, GC_ENOMEM, "cannot allocate the training workspace for %lld rows", (long long)cap);
    if (m.ws) dfree(ctx, m.ws);
    m.ws = mem;
    m.ws_rows = cap;
    carve_ws(static_cast<char *>(mem), R, part, m.w);
    return GC_OK;
}

// ---------------------------------------------------------------------------
// Training workspace of gc_mlp_train_step_noalloc: a file-scope device array
// (each device that loads the library holds its own copy until the process
// ends), sized for kStaticPairs point pairs.  Host code never passes the
// array's name to a kernel (in host code it names a host-side stand-in): it
// uses the device address read once per device with hipGetSymbolAddress.
// ---------------------------------------------------------------------------
constexpr int64_t kStaticPairs = 2048;
constexpr size_t kStaticRows = 2 * kStaticPairs;
constexpr size_t kStaticPart = ws_part_floats(kStaticRows, std::min<size_t>(kTrainGroups, kStaticRows / kRowsPerGroup));
constexpr size_t kStaticBytes = ws_bytes(kStaticRows, kStaticPart);
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Once per device, with that device current (gc_create): the device address of scratch.
void scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_done[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
    g_scratch_done[device] = true;
}

gc_status check_mlp_points(gc_ctx *ctx, const double *pts, int64_t n, const double *out) {
    if (n < 0) return fail(ctx, GC_EINVAL, "n must be >= 0");
    if (n > 0x7FFFFF00ll) return fail(ctx, GC_EINVAL, "too many points (%lld)", (long long)n);
    if (n > 0 && (!pts || !out)) return fail(ctx, GC_EINVAL, "pts and out must be set");
    return GC_OK;
}

}  // namespace

extern "C" {

gc_status gc_mlp_set(gc_ctx *ctx, const gc_mlp_desc *d) {
    if (!ctx || !d) return GC_EINVAL;
    if (!ctx->have_field) return fail(ctx, GC_ESTATE, "gc_mlp_set before gc_load_field");
    for (int j = 0; j < kMlpFreq; ++j) {
        const double a = d->freq[j][0], b = d->freq[j][1], n = d->freq[j][2];
        if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(n))
            return fail(ctx, GC_EINVAL, "frequency %d is not finite", j);
        if (n != std::floor(n) || std::fabs(n) > 4096.0)
            return fail(ctx, GC_EINVAL, "n_%d must be an integer of magnitude <= 4096 (got %g)", j, n);
    }
    if (!(d->r_ref > 0.0) || !std::isfinite(d->r_ref)) return fail(ctx, GC_EINVAL, "r_ref must be finite and > 0");
    for (int c = 0; c < kMlpOut; ++c)
        if (!std::isfinite(d->scale[c]) || !std::isfinite(d->power[c]))
            return fail(ctx, GC_EINVAL, "scale and power must be finite");
    if (d->params)
        for (int i = 0; i < kUserParams; ++i)
            if (!std::isfinite(d->params[i])) return fail(ctx, GC_EINVAL, "parameter %d is not finite", i);
    HIPCHK(hipSetDevice(ctx->opt.device));
    MlpState &m = ctx->mlp;
    hipStream_t s = ctx->stream;
    const size_t nw = (size_t)kMlpDepth * kMlpWidth * kMlpWidth;
    const size_t fbytes = align256((size_t)kMlpParams * 4);
    const size_t total = 4 * fbytes + 3 * align256(nw * 2) + align256((size_t)kMlpOutPad * kMlpWidth * 2) +
                         align256((size_t)kMlpEvalRows * kMlpWidth * 2);
    if (!m.mem) {
        if (dalloc(ctx, (void **)&m.mem, total) != hipSuccess) return fail(ctx, GC_ENOMEM, "cannot allocate the network");
        char *c = static_cast<char *>(m.mem);
        m.p = reinterpret_cast<float *>(c); c += fbytes;
        m.mo = reinterpret_cast<float *>(c); c += fbytes;
        m.ve = reinterpret_cast<float *>(c); c += fbytes;
        m.g = reinterpret_cast<float *>(c); c += fbytes;
        m.W = reinterpret_cast<__bf16 *>(c); c += align256(nw * 2);
        m.WT = reinterpret_cast<__bf16 *>(c); c += align256(nw * 2);
        m.We = reinterpret_cast<__bf16 *>(c); c += align256(nw * 2);
        m.Wo = reinterpret_cast<__bf16 *>(c); c += align256((size_t)kMlpOutPad * kMlpWidth * 2);
        m.Woe = reinterpret_cast<__bf16 *>(c);
    }
    std::vector<float> host;
    to_device_layout(d->params, host);
    HIPCHK(hipMemcpyAsync(m.p, host.data(), (size_t)kMlpParams * 4, hipMemcpyHostToDevice, s));
    for (float *z : {m.mo, m.ve, m.g}) HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(z), 0u, kMlpParams, s));
    HIPCHK(mlp_launch_refresh(m.p, m.W, m.WT, m.Wo, m.We, m.Woe, s));
    MlpArgs &a = m.args;
    a = MlpArgs{};
    a.W = m.We;
    a.Wo = m.Woe;
    a.c = m.p + kMlpOffC;
    a.co = m.p + kMlpOffCo;
    for (int j = 0; j < kMlpFreq; ++j) {
        a.fa[j] = (float)d->freq[j][0];
        a.fb[j] = (float)d->freq[j][1];
        a.fn[j] = (float)d->freq[j][2];
    }
    const double r_span = (double)(ctx->f.nr - 1) / ctx->f.inv_dr;
    a.r_min = (float)ctx->f.r_min;
    a.inv_rspan = (float)(1.0 / r_span);
    a.r_ref = (float)d->r_ref;
    for (int c = 0; c < kMlpOut; ++c) {
        a.scale[c] = (float)d->scale[c];
        a.power[c] = (float)d->power[c];
    }
    HIPCHK(hipStreamSynchronize(s));
    m.set = true;
    if (ctx->gexec) {
        (void)hipGraphExecDestroy(ctx->gexec);
        ctx->gexec = nullptr;
    }
    return GC_OK;
}

static gc_status mlp_copy_out(gc_ctx *ctx, const float *src, float *host_out) {
    if (!ctx) return GC_EINVAL;
    if (!host_out) return fail(ctx, GC_EINVAL, "host_out is NULL");
    if (!ctx->mlp.set) return fail(ctx, GC_ESTATE, "no neural field (gc_mlp_set)");
    HIPCHK(hipSetDevice(ctx->opt.device));
    std::vector<float> host(kMlpParams);
    HIPCHK(hipMemcpyAsync(host.data(), src, (size_t)kMlpParams * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    to_user_layout(host, host_out);
    return GC_OK;
}

gc_status gc_mlp_get_params(gc_ctx *ctx, float *host_out) {
    return mlp_copy_out(ctx, ctx ? ctx->mlp.p : nullptr, host_out);
}

gc_status gc_mlp_get_grads(gc_ctx *ctx, float *host_out) {
    return mlp_copy_out(ctx, ctx ? ctx->mlp.g : nullptr, host_out);
}

}  // extern "C"

namespace {

gc_status check_train(gc_ctx *ctx, const double *pts, const double *tgt, int64_t n_pairs, const gc_mlp_train_opts *o,
                      int64_t max_pairs) {
    if (!ctx->mlp.set) return fail(ctx, GC_ESTATE, "no neural field (gc_mlp_set)");
    if (n_pairs <= 0 || n_pairs > max_pairs)
        return fail(ctx, GC_EINVAL, "n_pairs must be in [1, %lld] (got %lld)", (long long)max_pairs, (long long)n_pairs);
    if (!pts || !tgt) return fail(ctx, GC_EINVAL, "pts and tgt must be set");
    if (o->apply && (o->step < 1 || !(o->lr > 0.0) || !(o->beta1 >= 0.0 && o->beta1 < 1.0) ||
                     !(o->beta2 >= 0.0 && o->beta2 < 1.0) || !(o->eps > 0.0)))
        return fail(ctx, GC_EINVAL, "Adam needs step >= 1, lr > 0, 0 <= beta1, beta2 < 1 and eps > 0");
    if (!(o->beta_pair >= 0.0) || !std::isfinite(o->beta_pair)) return fail(ctx, GC_EINVAL, "beta_pair must be >= 0");
    return GC_OK;
}

// Forward, loss, backward and the optional Adam update on the workspace w
// (which holds at least 2 n_pairs rows); the loss partials are read back.
gc_status train_step(gc_ctx *ctx, const double *pts, const double *tgt, int64_t n_pairs, const gc_mlp_train_opts *o,
                     double *loss, const TrainWs &w) {
    MlpState &m = ctx->mlp;
    hipStream_t s = ctx->stream;
    const int rows = (int)(2 * n_pairs);
    const size_t RW = (size_t)rows * kMlpWidth, WW = (size_t)kMlpWidth * kMlpWidth;
    // forward: H0 = features, H_{l+1} = silu(H_l W_l^T + c_l), Y = H6 W_o^T + c_o
    HIPCHK(mlp_launch_features(m.args, pts, rows, w.H, s));
    for (int l = 0; l < kMlpDepth; ++l)
        HIPCHK(mlp_launch_forward_layer(w.H + l * RW, m.W + l * WW, m.p + kMlpOffC + l * kMlpWidth, rows, w.Z + l * RW,
                                        w.H + (l + 1) * RW, s));
    HIPCHK(mlp_launch_output(w.H + kMlpDepth * RW, m.Wo, m.p + kMlpOffCo, rows, w.Y, s));
    // loss and its gradient with respect to the outputs
    MlpLoss L{};
    for (int c = 0; c < kMlpOut; ++c) L.wc[c] = o->wc[c];
    L.beta = o->beta_pair;
    const int lb = (int)std::min<int64_t>(kLossBlocks, (n_pairs + 255) / 256);
    HIPCHK(mlp_launch_loss(m.args, pts, tgt, w.Y, (int)n_pairs, L, w.dY, w.loss_part, lb, s));
    // backward; weight-gradient products split over row groups of about kRowsPerGroup rows
    const int groups = std::max(1, std::min(kTrainGroups, rows / kRowsPerGroup));
    HIPCHK(mlp_launch_out_grad(w.dY, w.H + kMlpDepth * RW, rows, w.part, m.g + kMlpOffWo, m.g + kMlpOffCo, s));
    HIPCHK(mlp_launch_out_back(w.dY, m.p + kMlpOffWo, rows, w.dH, s));
    for (int l = kMlpDepth - 1; l >= 0; --l) {
        HIPCHK(mlp_launch_dz(w.dH, w.Z + l * RW, rows, w.dZ, w.part, m.g + kMlpOffC + l * kMlpWidth, s));
        HIPCHK(mlp_launch_wgrad(w.dZ, w.H + l * RW, rows, groups, w.part, m.g + kMlpOffW + l * WW, s));
        if (l > 0) HIPCHK(mlp_launch_backward_data(w.dZ, m.WT + l * WW, rows, w.dH, s));
    }
    if (o->apply) {
        HIPCHK(mlp_launch_adam(m.p, m.mo, m.ve, m.g, kMlpParams, (float)o->lr, (float)o->beta1, (float)o->beta2,
                               (float)o->eps, o->step, s));
        HIPCHK(mlp_launch_refresh(m.p, m.W, m.WT, m.Wo, m.We, m.Woe, s));
    }
    double lp[kLossBlocks];
    HIPCHK(hipMemcpyAsync(lp, w.loss_part, lb * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double sum = 0.0;
    for (int i = 0; i < lb; ++i) sum += lp[i];
    if (loss) *loss = sum;
    return GC_OK;
}

}  // namespace

extern "C" {

gc_status gc_mlp_train_step(gc_ctx *ctx, const double *pts, const double *tgt, int64_t n_pairs,
                            const gc_mlp_train_opts *o, double *loss) {
    if (!ctx || !o) return GC_EINVAL;
    gc_status st = check_train(ctx, pts, tgt, n_pairs, o, 1 << 26);
    if (st != GC_OK) return st;
    HIPCHK(hipSetDevice(ctx->opt.device));
    st = mlp_workspace(ctx, 2 * n_pairs);
    if (st != GC_OK) return st;
    return train_step(ctx, pts, tgt, n_pairs, o, loss, ctx->mlp.w);
}

gc_status gc_mlp_train_step_noalloc(gc_ctx *ctx, const double *pts, const double *tgt, int64_t n_pairs,
                                    const gc_mlp_train_opts *o, double *loss) {
    if (!ctx || !o) return GC_EINVAL;
    gc_status st = check_train(ctx, pts, tgt, n_pairs, o, kStaticPairs);
    if (st != GC_OK) return st;
    const int dev = ctx->opt.device;
    if (dev < 0 || dev >= kMaxDevices || !g_scratch_done[dev])
        return fail(ctx, GC_EDEVICE, "no static workspace on device %d", dev);
    if (!g_scratch_ptr[dev])
        return fail(ctx, GC_EDEVICE, "static workspace of device %d: %s", dev, hipGetErrorString(g_scratch_err[dev]));
    HIPCHK(hipSetDevice(dev));
    TrainWs w{};
    carve_ws(static_cast<char *>(g_scratch_ptr[dev]), kStaticRows, kStaticPart, w);
    return train_step(ctx, pts, tgt, n_pairs, o, loss, w);
}

gc_status gc_mlp_eval(gc_ctx *ctx, const double *pts, int64_t n, double *out) {
    if (!ctx) return GC_EINVAL;
    if (!ctx->mlp.set) return fail(ctx, GC_ESTATE, "no neural field (gc_mlp_set)");
    gc_status st = check_mlp_points(ctx, pts, n, out);
    if (st != GC_OK || n == 0) return st;
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(mlp_launch_eval(ctx->mlp.args, pts, (int)n, out, ctx->stream));
    return GC_OK;
}

gc_status gc_field_sample(gc_ctx *ctx, const double *pts, int64_t n, double *out) {
    if (!ctx) return GC_EINVAL;
    if (!ctx->have_field) return fail(ctx, GC_ESTATE, "gc_field_sample before gc_load_field");
    gc_status st = check_mlp_points(ctx, pts, n, out);
    if (st != GC_OK || n == 0) return st;
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(launch_field_sample(ctx->f, pts, (int)n, out, ctx->stream));
    return GC_OK;
}

}  // extern "C"
