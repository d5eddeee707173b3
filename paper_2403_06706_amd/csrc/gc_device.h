// gc_device.h -- device building blocks of the push: counter-based random
// numbers, trilinear field gather, guiding-centre right-hand side.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "gc_internal.h"

namespace gc {

constexpr double kC = 299792458.0;                    // speed of light (m/s)
constexpr double kInvC2 = 1.0 / (299792458.0 * 299792458.0);
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of the
// 64x64->128-bit multiply-xor bijection, key advanced by two Weyl constants.
// ---------------------------------------------------------------------------
struct U64x4 { uint64_t v[4]; };

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round) { k0 += 0x9E3779B97F4A7C15ULL; k1 += 0xBB67AE8584CAA73BULL; }
        const uint64_t m0 = 0xD2E7470EE14C6C93ULL, m1 = 0xCA5A826395121157ULL;
        uint64_t hi0 = __umul64hi(m0, c0), lo0 = m0 * c0;
        uint64_t hi1 = __umul64hi(m1, c2), lo1 = m1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    U64x4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// uniform double on [0, 1) from the top 53 bits
__device__ __forceinline__ double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// counter word 2: what the block is drawn for
enum : uint64_t { kPurposePath = 0, kPurposeInject = 1 };

// ---------------------------------------------------------------------------
// Trilinear interpolation of the packed grid in index space: r nodes from
// r_min with spacing dr, theta nodes at (j + 1/2) dth, phi periodic.  The
// stencil is clamped to the grid in floating point before any conversion to
// an integer, so every load stays inside the buffer for any input.
// Returns false if the input or any interpolated value is not finite.
//
// The packed layout (chunks of W components, 4 x 2 node blocks) is described
// with field_layout in gc_internal.h.  Loads address the field as its base
// (uniform, or plus a uniform chunk offset) and a 32-bit byte offset per lane,
// the form of the SGPR-base global load; the packed field is at most 4 GiB.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R clampr(R x, R lo, R hi) { return fmin(fmax(x, lo), hi); }

// Chunk width and count per node of each storage type (as field_layout).
template <int FDT> struct Layout { static constexpr uint32_t W = 4, nch = 3; };   // FP32, FP16
template <> struct Layout<GC_F64> { static constexpr uint32_t W = 2, nch = 6; };

template <int FDT> struct Pair;   // 24 values of two phi-adjacent nodes, 12 components each

// Each load(): off = element offset of chunk 0 of the pair's first node, dk =
// offset of the second node from the first, cs = element stride between
// chunks; chunk c of node h is at off + h dk + c cs.
template <> struct Pair<GC_F32> {
    float v[24];
    __device__ __forceinline__ void load(const void *base, uint32_t off, uint32_t dk, uint32_t cs) {
        const char *b = static_cast<const char *>(base);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const float4 x = *reinterpret_cast<const float4 *>(b + (size_t)((q % 3) * cs) * 4u +
                                                               (off + (q / 3) * dk) * 4u);
            v[4 * q + 0] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
        }
    }
    __device__ __forceinline__ float get(int c, const FieldDev &) const { return v[c]; }
};

template <> struct Pair<GC_F64> {
    double v[24];
    __device__ __forceinline__ void load(const void *base, uint32_t off, uint32_t dk, uint32_t cs) {
        const char *b = static_cast<const char *>(base);
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            const double2 x = *reinterpret_cast<const double2 *>(b + (size_t)((q % 6) * cs) * 8u +
                                                                (off + (q / 6) * dk) * 8u);
            v[2 * q + 0] = x.x; v[2 * q + 1] = x.y;
        }
    }
    __device__ __forceinline__ double get(int c, const FieldDev &) const { return v[c]; }
};

template <> struct Pair<GC_F16> {
    __half v[24];
    __device__ __forceinline__ void load(const void *base, uint32_t off, uint32_t dk, uint32_t cs) {
        const char *b = static_cast<const char *>(base);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const uint2 x = *reinterpret_cast<const uint2 *>(b + (size_t)((q % 3) * cs) * 2u +
                                                             (off + (q / 3) * dk) * 2u);
            __half h[4];
            __builtin_memcpy(h, &x, 8);
            v[4 * q + 0] = h[0]; v[4 * q + 1] = h[1]; v[4 * q + 2] = h[2]; v[4 * q + 3] = h[3];
        }
    }
    __device__ __forceinline__ float get(int c, const FieldDev &f) const {
        return __half2float(v[c]) * f.scale[c % 12];
    }
};

// Stencil of a trilinear gather: the four node pairs (r, theta corners, each
// with its two phi nodes) and their weights.
template <typename R>
struct GatherPlan {
    R w[4];              // (r, theta) weight of each node pair
    R wp;                // phi weight of the second node of a pair
    uint32_t off[4];     // element offset of chunk 0 of each pair's first node
    uint32_t dk;         // offset of a pair's second (phi) node from its first
    uint32_t cs;         // element stride between chunks
    uint32_t rec;        // element offset of the first node of pair 0 in the node records
};

template <int FDT, typename R>
__device__ __forceinline__ bool gather_plan(const FieldDev &f, R r, R th, R ph, GatherPlan<R> &gp) {
    R x = (r - (R)f.r_min) * (R)f.inv_dr;
    R y = th * (R)f.inv_dth - (R)0.5;
    R z = ph * (R)f.inv_dph;
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) return false;
    const R nph = (R)f.nph;
    R fi = clampr(floor(x), (R)0, (R)(f.nr - 2));
    R fj = clampr(floor(y), (R)0, (R)(f.nth - 2));
    R wr = clampr(x - fi, (R)0, (R)1);
    R wt = clampr(y - fj, (R)0, (R)1);
    R zf = floor(z);
    gp.wp = z - zf;
    R km = zf - nph * floor(zf * (R)f.inv_nph);
    km = km < (R)0 ? km + nph : km;
    km = km >= nph ? km - nph : km;
    km = clampr(km, (R)0, nph - (R)1);
    const uint32_t i = (uint32_t)fi, j = (uint32_t)fj, k = (uint32_t)km;
    constexpr uint32_t W = Layout<FDT>::W;
    // separable offsets of the blocked layout (field_layout)
    const uint32_t i1 = i + 1u;
    const uint32_t gi0 = (i >> 2) * (kLayB * W) + (i & 3u) * W;
    const uint32_t gi1 = (i1 >> 2) * (kLayB * W) + (i1 & 3u) * W;
    const uint32_t gk0 = (k >> 1) * f.ks + (k & 1u) * (kLayBr * W);
    gp.dk = (k & 1u) ? f.ks - kLayBr * W : kLayBr * W;          // gK(k + 1) - gK(k)
    const uint32_t gj0 = j * f.js;
    gp.cs = f.cs;
    gp.rec = ((i * (uint32_t)f.nth + j) * (uint32_t)(f.nph + 1) + k) * 12u;
    gp.w[0] = ((R)1 - wr) * ((R)1 - wt);
    gp.w[1] = ((R)1 - wr) * wt;
    gp.w[2] = wr * ((R)1 - wt);
    gp.w[3] = wr * wt;
    gp.off[0] = gj0 + gk0 + gi0;
    gp.off[1] = gj0 + f.js + gk0 + gi0;
    gp.off[2] = gj0 + gk0 + gi1;
    gp.off[3] = gj0 + f.js + gk0 + gi1;
    return true;
}

// Add node pair p (index q of the stencil) to out: for each component,
// out = fma(wb, B, fma(wa, A, out)) with wa = w_q (1 - w_ph), wb = w_q w_ph.
template <int FDT, typename R>
__device__ __forceinline__ void gather_add(const FieldDev &f, const GatherPlan<R> &gp, int q, const Pair<FDT> &p,
                                           R out[12]) {
    const R wa = gp.w[q] * ((R)1 - gp.wp), wb = gp.w[q] * gp.wp;
#pragma unroll
    for (int c = 0; c < 12; ++c) out[c] = fma(wb, (R)p.get(c + 12, f), fma(wa, (R)p.get(c, f), out[c]));
}

template <typename R>
__device__ __forceinline__ bool finite12(const R out[12]) {
    R sum = (R)0;
#pragma unroll
    for (int c = 0; c < 12; ++c) sum += out[c];
    return isfinite(sum);
}

// One lane: the four node pairs added in order.
// kAllPairs: issue the loads of all four node pairs at once (one memory round
// trip per gather, more registers); otherwise at most two pairs are in
// registers at a time, which keeps the push within two wavefronts per SIMD.
// The arithmetic, and so the result, is the same either way.  kTame: the
// caller knows the field is tame (FieldDev::tame): no finiteness test.
template <int FDT, typename R, bool kAllPairs = false, bool kTame = false>
__device__ __forceinline__ bool gather(const FieldDev &f, R r, R th, R ph, R out[12]) {
    GatherPlan<R> gp;
    if (!gather_plan<FDT>(f, r, th, ph, gp)) return false;
#pragma unroll
    for (int c = 0; c < 12; ++c) out[c] = (R)0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        Pair<FDT> p;
        p.load(f.data, gp.off[q], gp.dk, gp.cs);
        gather_add<FDT, R>(f, gp, q, p, out);
        if (!kAllPairs && (q & 1)) __builtin_amdgcn_sched_barrier(0);   // at most two node pairs in registers
    }
    if constexpr (kTame) return true;
    else return finite12(out);
}

// The field and the extra node array of the full Eqs. 1-2 (same geometry and
// layout, fx the extra array's description) at one point, with one stencil:
// the same operations and order as gather() on each array.  Returns what
// gather() returns for the field; xok what it returns for the extra array.
template <int FDT, typename R, bool kAllPairs = false>
__device__ __forceinline__ bool gather2(const FieldDev &f, const FieldDev &fx, R r, R th, R ph, R out[12],
                                        R xout[12], bool &xok) {
    GatherPlan<R> gp;
    xok = false;
    if (!gather_plan<FDT>(f, r, th, ph, gp)) return false;
#pragma unroll
    for (int c = 0; c < 12; ++c) out[c] = xout[c] = (R)0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        Pair<FDT> p;
        p.load(f.data, gp.off[q], gp.dk, gp.cs);
        gather_add<FDT, R>(f, gp, q, p, out);
        if (!kAllPairs && (q & 1)) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        Pair<FDT> p;
        p.load(fx.data, gp.off[q], gp.dk, gp.cs);
        gather_add<FDT, R>(fx, gp, q, p, xout);
        if (!kAllPairs && (q & 1)) __builtin_amdgcn_sched_barrier(0);
    }
    xok = finite12(xout);
    return finite12(out);
}

// Word j of lane J of an aligned group of four lanes, to every lane of the
// group (DPP quad permutation [J, J, J, J]).
template <int J>
__device__ __forceinline__ uint32_t quad_bcast(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, J * 0x55, 0xF, 0xF, false);
}

template <int FDT, int J>
__device__ __forceinline__ Pair<FDT> quad_bcast_pair(const Pair<FDT> &mine) {
    constexpr int kWords = sizeof(Pair<FDT>) / 4;
    static_assert(sizeof(Pair<FDT>) % 4 == 0, "pair storage must be whole words");
    uint32_t w[kWords];
    __builtin_memcpy(w, &mine, sizeof w);
#pragma unroll
    for (int i = 0; i < kWords; ++i) w[i] = quad_bcast<J>(w[i]);
    Pair<FDT> p;
    __builtin_memcpy(&p, w, sizeof w);
    return p;
}

// A value of lane J of an aligned quad, to every lane of the quad.
template <int J, typename R>
__device__ __forceinline__ R quad_bcast_value(R x) {
    static_assert(sizeof(R) % 4 == 0, "whole words");
    uint32_t w[sizeof(R) / 4];
    __builtin_memcpy(w, &x, sizeof w);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(R) / 4); ++i) w[i] = quad_bcast<J>(w[i]);
    R y;
    __builtin_memcpy(&y, w, sizeof w);
    return y;
}

// Four lanes of an aligned quad, one particle (FP32 and FP64 fields), on the
// node records f.rec: lane gl loads components 3gl..3gl+2 of both nodes of the
// four node pairs (a pair's nodes are adjacent records, 48 or 96 bytes each),
// runs their chains with the operations and order of gather_add, and the quad
// exchanges the finished components, so all four lanes hold the bits of
// gather().  Each lane converts and multiplies a quarter of the values.  All
// four lanes must call it together.
template <int FDT, typename R, bool kTame = false>
__device__ __forceinline__ bool gather_quad_split(const FieldDev &f, R r, R th, R ph, uint32_t gl, R out[12]) {
    using T = typename std::conditional<FDT == GC_F64, double, float>::type;
    GatherPlan<R> gp;
    if (!gather_plan<FDT>(f, r, th, ph, gp)) return false;
    const uint32_t row = (uint32_t)(f.nph + 1) * 12u;                 // theta stride of the records
    const uint32_t o[4] = {gp.rec, gp.rec + row, gp.rec + (uint32_t)f.nth * row,
                           gp.rec + (uint32_t)f.nth * row + row};     // the pairs, in gather_add's order
    // per-lane 64-bit addresses: the three components of a node merge into one
    // load and the second node is a constant offset from the first
    const T *base = static_cast<const T *>(f.rec) + 3u * gl;
    T v[4][6];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const T *p = base + o[q];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[q][c] = p[c];            // node k
            v[q][3 + c] = p[12 + c];   // node k + 1
        }
    }
    R acc[3] = {(R)0, (R)0, (R)0};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const R wa = gp.w[q] * ((R)1 - gp.wp), wb = gp.w[q] * gp.wp;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = fma(wb, (R)v[q][3 + c], fma(wa, (R)v[q][c], acc[c]));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        out[c] = quad_bcast_value<0>(acc[c]);
        out[3 + c] = quad_bcast_value<1>(acc[c]);
        out[6 + c] = quad_bcast_value<2>(acc[c]);
        out[9 + c] = quad_bcast_value<3>(acc[c]);
    }
    if constexpr (kTame) return true;
    else return finite12(out);
}

// Four lanes of an aligned quad, one particle: for FP32 and FP64 fields the
// component split above; for FP16 fields lane gl loads node pair gl, the quad
// shares the loaded words, and every lane adds the four pairs in the one-lane
// order.  Either way all four lanes hold the bits of gather().  All four lanes
// must call it together.
template <int FDT, typename R, bool kTame = false>
__device__ __forceinline__ bool gather_quad(const FieldDev &f, R r, R th, R ph, uint32_t gl, R out[12]) {
    if constexpr (FDT != GC_F16) return gather_quad_split<FDT, R, kTame>(f, r, th, ph, gl, out);
    GatherPlan<R> gp;
    if (!gather_plan<FDT>(f, r, th, ph, gp)) return false;
    Pair<FDT> mine;
    mine.load(f.data, gp.off[gl], gp.dk, gp.cs);
#pragma unroll
    for (int c = 0; c < 12; ++c) out[c] = (R)0;
    gather_add<FDT, R>(f, gp, 0, quad_bcast_pair<FDT, 0>(mine), out);
    gather_add<FDT, R>(f, gp, 1, quad_bcast_pair<FDT, 1>(mine), out);
    gather_add<FDT, R>(f, gp, 2, quad_bcast_pair<FDT, 2>(mine), out);
    gather_add<FDT, R>(f, gp, 3, quad_bcast_pair<FDT, 3>(mine), out);
    if constexpr (kTame) return true;
    else return finite12(out);
}

// ---------------------------------------------------------------------------
// Reciprocal, inverse square root and sine for the right-hand side.
// Hardware estimates refined by Newton steps (two in double, one in float:
// each step doubles the correct bits), faithful to about one ulp for the
// normal, finite arguments met here.  sin on [0, pi] (theta of a particle
// inside the grid) folds to [0, pi/4] and sums the Taylor series of sin or
// cos up to the z^17 / z^16 term (truncation below 1e-19).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float rcp_nr(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx, y * y, 1.5);
    return y * fma(-hx, y * y, 1.5);
}
__device__ __forceinline__ float rsqrt_nr(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    return y * fmaf(-0.5f * x, y * y, 1.5f);
}

template <typename R>
__device__ __forceinline__ R sin_0_pi(R x) {
    const R half_pi = (R)1.5707963267948966, pi = (R)3.141592653589793, quarter_pi = (R)0.7853981633974483;
    const R y = x > half_pi ? pi - x : x;            // sin(x) = sin(pi - x)
    const bool use_cos = y > quarter_pi;
    const R z = use_cos ? half_pi - y : y;           // sin(y) = cos(pi/2 - y)
    const R z2 = z * z;
    // One series per lane, behind a branch: the particles of a wavefront are
    // binned by cell, so nearly always all of its lanes take the same one.
    if (use_cos) {
        // cos z = 1 - z^2/2! + z^4/4! - ... + z^16/16!
        R pc = (R)(1.0 / 20922789888000.0);
        pc = fma(pc, -z2, (R)(1.0 / 87178291200.0));
        pc = fma(pc, -z2, (R)(1.0 / 479001600.0));
        pc = fma(pc, -z2, (R)(1.0 / 3628800.0));
        pc = fma(pc, -z2, (R)(1.0 / 40320.0));
        pc = fma(pc, -z2, (R)(1.0 / 720.0));
        pc = fma(pc, -z2, (R)(1.0 / 24.0));
        pc = fma(pc, -z2, (R)0.5);
        return fma(pc, -z2, (R)1);
    }
    // sin z = z (1 - z^2/3! + z^4/5! - ... + z^16/17!)
    R ps = (R)(1.0 / 355687428096000.0);
    ps = fma(ps, -z2, (R)(1.0 / 1307674368000.0));
    ps = fma(ps, -z2, (R)(1.0 / 6227020800.0));
    ps = fma(ps, -z2, (R)(1.0 / 39916800.0));
    ps = fma(ps, -z2, (R)(1.0 / 362880.0));
    ps = fma(ps, -z2, (R)(1.0 / 5040.0));
    ps = fma(ps, -z2, (R)(1.0 / 120.0));
    ps = fma(ps, -z2, (R)(1.0 / 6.0));
    ps = fma(ps, -z2, (R)1);
    return z * ps;
}

// ---------------------------------------------------------------------------
// Guiding-centre right-hand side, Eqs. (1)-(2), reduced to the terms the
// twelve gridded components determine (b, E, grad|B|, (b.grad)b):
//   gamma = sqrt(1 + (u^2 + 2 mu B)/c^2)      (mu = mu_B / m, u = gamma v_par)
//   dR/dt = v_par b + v_E + (gamma/(q/m B)) b x a,
//   a     = (mu/gamma^2) grad B + ((q/m) v_par E_par/(gamma c^2)) v_E + v_par^2 (b.grad)b
//   du/dt = (q/m) E_par - (mu/gamma) b.grad B + gamma v_par v_E.(b.grad)b
// drift-free form (only v_par b kept): dR/dt = v_par b, du/dt without the v_E term.
// Output: coordinate rates (dr/dt, dth/dt, dph/dt, du/dt) and v_par.
// kFull: the full Eqs. 1-2, x = (v_E.grad)b, (b.grad)v_E, (v_E.grad)v_E at the
// point: v_par (x0..2 + x3..5) + x6..8 joins the bracket of dR/dt and
// gamma v_E.x0..2 joins du/dt.
// ---------------------------------------------------------------------------
template <typename R, bool kFull = false>
__device__ __forceinline__ void gc_rhs(R r, R th, R u, R mu, R qm, R iqm, bool drift_free,
                                       const R g[12], R F[4], R &vpar, const R *x = nullptr) {
    const R Bx = g[0], By = g[1], Bz = g[2];
    const R Ex = g[3], Ey = g[4], Ez = g[5];
    const R Gx = g[6], Gy = g[7], Gz = g[8];
    const R Kx = g[9], Ky = g[10], Kz = g[11];
    const R B2 = Bx * Bx + By * By + Bz * Bz;
    const R iB = rsqrt_nr(B2);
    const R B = B2 * iB;
    const R bx = Bx * iB, by = By * iB, bz = Bz * iB;
    const R g2 = (R)1 + (u * u + (R)2 * mu * B) * (R)kInvC2;
    const R ig = rsqrt_nr(g2);
    const R gamma = g2 * ig;
    vpar = u * ig;
    const R Epar = Ex * bx + Ey * by + Ez * bz;
    const R vEx = (Ey * bz - Ez * by) * iB;
    const R vEy = (Ez * bx - Ex * bz) * iB;
    const R vEz = (Ex * by - Ey * bx) * iB;
    const R bG = bx * Gx + by * Gy + bz * Gz;
    R Vx, Vy, Vz, udot;
    if (drift_free) {
        Vx = vpar * bx; Vy = vpar * by; Vz = vpar * bz;
        udot = qm * Epar - mu * ig * bG;
    } else {
        const R cG = mu * ig * ig;
        const R cE = qm * vpar * Epar * ig * (R)kInvC2;
        const R cK = vpar * vpar;
        R ax = cG * Gx + cE * vEx + cK * Kx;
        R ay = cG * Gy + cE * vEy + cK * Ky;
        R az = cG * Gz + cE * vEz + cK * Kz;
        if (kFull) {
            ax += vpar * (x[0] + x[3]) + x[6];
            ay += vpar * (x[1] + x[4]) + x[7];
            az += vpar * (x[2] + x[5]) + x[8];
        }
        const R pref = gamma * iqm * iB;
        Vx = vpar * bx + vEx + pref * (by * az - bz * ay);
        Vy = vpar * by + vEy + pref * (bz * ax - bx * az);
        Vz = vpar * bz + vEz + pref * (bx * ay - by * ax);
        udot = qm * Epar - mu * ig * bG + gamma * vpar * (vEx * Kx + vEy * Ky + vEz * Kz);
        if (kFull) udot += gamma * (vEx * x[0] + vEy * x[1] + vEz * x[2]);
    }
    const R ir = rcp_nr(r);
    F[0] = Vx;
    F[1] = Vy * ir;
    F[2] = Vz * ir * rcp_nr(sin_0_pi(th));
    F[3] = udot;
}

}  // namespace gc
