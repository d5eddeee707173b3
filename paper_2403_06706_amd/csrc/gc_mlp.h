// gc_mlp.h -- neural field: a Fourier-feature MLP that replaces the gridded
// field, evaluated with BF16 matrix-core (MFMA) instructions, FP32 accumulation.
//
//   x~ = ((r - r_min)/(r_max - r_min), th/pi),  psi_j = 2 pi (a_j r~ + b_j th~) + n_j ph,  j < 64
//   h0 = [sin psi_0, cos psi_0, sin psi_1, ...]       (128 features, n_j integer: periodic in ph)
//   h_l = silu(W_l h_{l-1} + c_l), l = 1..6;  y = W_o h_6 + c_o  (6 outputs)
//   B_i = S_i (r_ref/r)^p_i y_i,  E_i = S_{i+3} (r_ref/r)^p_{i+3} y_{i+3}
// grad|B| and (b.grad)b come from the derivatives of B along (r, th, ph),
// propagated forward through the network as three tangents, with the metric
// factors and connection terms of the local spherical basis.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gc {

constexpr int kMlpFreq = 64;
constexpr int kMlpWidth = 128;
constexpr int kMlpDepth = 6;
constexpr int kMlpOut = 6;
constexpr int kMlpOutPad = 32;     // output layer padded to one 32-wide MFMA tile
// fp32 parameter block: W[6][128][128] | c[6][128] | Wo[32][128] | co[32]
constexpr int kMlpOffW = 0;
constexpr int kMlpOffC = kMlpDepth * kMlpWidth * kMlpWidth;
constexpr int kMlpOffWo = kMlpOffC + kMlpDepth * kMlpWidth;
constexpr int kMlpOffCo = kMlpOffWo + kMlpOutPad * kMlpWidth;
constexpr int kMlpParams = kMlpOffCo + kMlpOutPad;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

// Everything an evaluation needs (passed by value to kernels).
struct MlpArgs {
    const __bf16 *W;      // [6][128][128] bf16 in evaluation order: row = output unit; the
                          // columns of layers 2..6 permuted within each 32-block (mlp_perm)
    const __bf16 *Wo;     // [16][128] bf16, columns permuted like W, rows >= 6 zero
    const float *c;       // [6][128]
    const float *co;      // [32]
    float fa[kMlpFreq], fb[kMlpFreq], fn[kMlpFreq];   // frequencies a_j, b_j, n_j
    float r_min, inv_rspan, r_ref;
    float scale[kMlpOut], power[kMlpOut];
};
constexpr int kMlpEvalRows = 16;   // rows of the evaluation copy of the output layer

// Column order of the evaluation weights of layers 2..6 and of the output
// layer: slot kappa of a 32-column block holds the weight of hidden unit
// mlp_perm(kappa) of that block.  With it, the hidden units a lane holds after
// one layer (the 16x16 accumulator layout) are exactly the input slots it must
// supply to the next (the B-operand layout), so activations never leave the
// registers.
__host__ __device__ constexpr int mlp_perm(int kappa) {
    return 16 * ((kappa & 7) >> 2) + 4 * (kappa >> 3) + (kappa & 3);
}

__device__ __forceinline__ float sigmoid_f(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_f(float z) { return z * sigmoid_f(z); }
__device__ __forceinline__ float dsilu_f(float z) {
    const float s = sigmoid_f(z);
    return s * (1.0f + z * (1.0f - s));
}

// The evaluation carries every hidden pre-activation and activation in log2
// units, z' = z log2(e) and h' = h log2(e) (the biases and the layer-1 inputs
// are scaled by log2(e), the output products by ln 2): then e^-z = 2^-z' is one
// hardware exp2, and the weights are used as stored.
constexpr float kMlpLog2e = 1.4426950408889634f, kMlpLn2 = 0.6931471805599453f;

// Workgroup LDS of the evaluation (NT threads): two staged weight matrices
// (rows padded to 144 BF16, 288 bytes: measured on the network push, the LDS
// bank-conflict cycles per conflict-free cycle are 0.08 with this pitch, 0.65
// with 136 and 4.1 with 128), the biases and frequencies, and each thread's
// outputs.
constexpr int kMlpLdsRowW = kMlpWidth + 16;
constexpr int kMlpLdsMat = kMlpWidth * kMlpLdsRowW;
constexpr int kMlpPieces = kMlpWidth * kMlpWidth / 8;       // 16-byte pieces of a 128 x 128 matrix
constexpr int kMlpOutPieces = kMlpEvalRows * kMlpWidth / 8; // of the 16-row output matrix
template <int NT>
struct MlpLds {
    __bf16 w[2][kMlpLdsMat];
    float c[kMlpDepth * kMlpWidth];
    float co[kMlpEvalRows];
    float fa[kMlpFreq], fb[kMlpFreq], fn[kMlpFreq];
    float y[NT][4 * kMlpOut];     // per thread: y, then dy along r, th, ph
};

// Biases and frequencies into LDS (all threads of the workgroup; followed by
// a barrier).
template <int NT>
__device__ __forceinline__ void mlp_lds_init(const MlpArgs &m, MlpLds<NT> &L) {
    for (int i = threadIdx.x; i < kMlpDepth * kMlpWidth; i += NT) L.c[i] = m.c[i] * kMlpLog2e;
    if (threadIdx.x < kMlpEvalRows) L.co[threadIdx.x] = threadIdx.x < kMlpOut ? m.co[threadIdx.x] : 0.0f;
    if (threadIdx.x < kMlpFreq) {
        L.fa[threadIdx.x] = m.fa[threadIdx.x];
        L.fb[threadIdx.x] = m.fb[threadIdx.x];
        L.fn[threadIdx.x] = m.fn[threadIdx.x];
    }
    __syncthreads();
}

// Pieces [U0, U0 + U) of this thread's share (piece u * NT + tid) of matrix mi
// (0..5 hidden layers, 6 output layer).  Branch-free: for the 16-row output
// matrix the surplus pieces repeat its last piece and land in rows that are
// never read.
template <int NT, int U0, int U>
__device__ __forceinline__ void mlp_fetch(const MlpArgs &m, int mi, u32x4 v[U]) {
    const bool hidden = mi < kMlpDepth;
    const u32x4 *src = reinterpret_cast<const u32x4 *>(hidden ? m.W + (size_t)mi * kMlpWidth * kMlpWidth : m.Wo);
    const int last = (hidden ? kMlpPieces : kMlpOutPieces) - 1;
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = src[min((U0 + u) * NT + (int)threadIdx.x, last)];
}

template <int NT, int U0, int U>
__device__ __forceinline__ void mlp_store(const u32x4 v[U], __bf16 *dst) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = (U0 + u) * NT + (int)threadIdx.x;
        *reinterpret_cast<u32x4 *>(dst + (e >> 4) * kMlpLdsRowW + (e & 15) * 8) = v[u];
    }
}

// Evaluate the network and its three tangents for the particles of an
// NT-thread workgroup (one per thread).  All NT threads must call it together
// (it synchronizes the workgroup); the biases must be in L (mlp_lds_init).
// Output per thread: y[6] and dy[d][6] = dy / d(r, th, ph)[d].
//
// Matrix-core tiling (v_mfma_f32_16x16x32_bf16; each wavefront takes its 64
// particles in 4 passes of 16): the products are taken transposed, Z^T = W H^T,
// so that the weights are the A operand and the activations the B operand.
// The B operand has four column tiles: the values of the 16 particles and
// their derivatives along r, th and ph.  In the 16x16 accumulator layout a lane
// then holds, for its particle column, the same hidden units in all four
// tiles: the activation (silu of the value, silu' times each tangent) is
// lane-local, and with the column permutation of the weights (mlp_perm) its
// results are already the next layer's B operand; activations never leave the
// registers.  The weights go through LDS, one matrix at a time, shared by the
// workgroup's wavefronts; the next matrix is fetched from global memory in two
// halves while the current one is in use.  Per pass and hidden layer: 8 unit
// tiles x 4 k-blocks x 4 column tiles = 128 MFMAs, the products of tile t
// issued before the activation of tile t - 1, which they overlap.
template <int NT, int kUnroll = 1>
__device__ __forceinline__ void mlp_block(const MlpArgs &m, float r, float th, float ph, MlpLds<NT> &L,
                                          float y[kMlpOut], float dy[3][kMlpOut]) {
    constexpr int kPer = kMlpPieces / NT;                  // pieces per thread
    constexpr int kHalf = kPer / 2;
    static_assert(kPer >= 2 && kPer % 2 == 0, "NT must divide the matrix into an even number of pieces");
    const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = l >> 4, col = l & 15;
    const float two_pi = 6.283185307179586f;
    float *yw = &L.y[wave * 64][0];                          // this wavefront's outputs
    u32x4 pf[kPer];
    __syncthreads();                                         // the previous call is done with both buffers
    mlp_fetch<NT, 0, kPer>(m, 0, pf);
    mlp_store<NT, 0, kPer>(pf, L.w[0]);
    int cur = 0;
    for (int p = 0; p < 4; ++p) {
        const int src = 16 * p + col;                        // the particle of this lane's column
        const float pr = __shfl(r, src), pth = __shfl(th, src), pph = __shfl(ph, src);
        const float rt = (pr - m.r_min) * m.inv_rspan, tt = pth * 0.3183098861837907f;
        // layer-1 inputs: features 32s + 8g + i (phases 16s + 4g + i/2), natural order
        bf16x8 B[4][4];                                      // [k block][value, d/dr, d/dth, d/dph]
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int i2 = 0; i2 < 4; ++i2) {
                const int j = 16 * s + 4 * g + i2;
                const float fa = L.fa[j], fb = L.fb[j], fn = L.fn[j];
                const float psi = two_pi * (fa * rt + fb * tt) + fn * pph;
                float sn, cs;
                __sincosf(psi, &sn, &cs);
                sn *= kMlpLog2e;                             // inputs in log2 units (see mlp_block)
                cs *= kMlpLog2e;
                const float dr = two_pi * fa * m.inv_rspan, dth = 2.0f * fb;
                B[s][0][2 * i2] = (__bf16)sn;
                B[s][0][2 * i2 + 1] = (__bf16)cs;
                B[s][1][2 * i2] = (__bf16)(cs * dr);
                B[s][1][2 * i2 + 1] = (__bf16)(-sn * dr);
                B[s][2][2 * i2] = (__bf16)(cs * dth);
                B[s][2][2 * i2 + 1] = (__bf16)(-sn * dth);
                B[s][3][2 * i2] = (__bf16)(cs * fn);
                B[s][3][2 * i2 + 1] = (__bf16)(-sn * fn);
            }
        }
        // kUnroll = kMlpDepth + 1 unrolls the layers: the next layer's operands
        // (Bn) and the current ones (B) then swap register sets instead of being
        // copied after every layer (measured: +9 % in the push, -7 % in the
        // plain evaluation kernel, which keeps the loop)
#pragma unroll(kUnroll)
        for (int mi = 0; mi <= kMlpDepth; ++mi) {
            __syncthreads();                                 // L.w[cur] holds matrix mi
            const int next = mi < kMlpDepth ? mi + 1 : 0;    // after the last: unused
            __bf16 *nbuf = L.w[cur ^ 1];
            const __bf16 *Wl = L.w[cur] + col * kMlpLdsRowW + 8 * g;
            if (mi < kMlpDepth) {
                bf16x8 Bn[4][4];
                const float *cl = L.c + mi * kMlpWidth + 4 * g;
                floatx4 prev[4];
#pragma unroll
                for (int t = 0; t <= 8; ++t) {
                    if (t == 0) mlp_fetch<NT, 0, kHalf>(m, next, pf);
                    if (t == 4) {
                        mlp_store<NT, 0, kHalf>(pf, nbuf);
                        mlp_fetch<NT, kHalf, kHalf>(m, next, pf);
                    }
                    // the value tile starts from the bias of its units (16t + 4g + jj)
                    floatx4 acc[4] = {floatx4{}, floatx4{}, floatx4{}, floatx4{}};
                    if (t < 8) {
                        acc[0] = *reinterpret_cast<const floatx4 *>(cl + 16 * t);
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(Wl + t * 16 * kMlpLdsRowW + 32 * s);
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, B[s][q], acc[q], 0, 0, 0);
                        }
                    }
                    if (t > 0) {
                        // lane holds units 16u + 4g + jj (u = t - 1): slots 8g + 4(u&1) + jj of k block u/2
                        const int u = t - 1;
                        // the four units side by side, one operation at a time, so that
                        // the transcendental latencies of the units overlap
                        float sg[4], h[4], ds[4];
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) sg[jj] = __builtin_amdgcn_exp2f(-prev[0][jj]);   // e^-z
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) sg[jj] = __builtin_amdgcn_rcpf(1.0f + sg[jj]);
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) h[jj] = prev[0][jj] * sg[jj];
                        // silu'(z) = s + z s (1 - s) = s + h' ln2 (1 - s)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) ds[jj] = fmaf(h[jj], fmaf(-kMlpLn2, sg[jj], kMlpLn2), sg[jj]);
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) {
                            const int s2 = u >> 1, i = (u & 1) * 4 + jj;
                            Bn[s2][0][i] = (__bf16)h[jj];
                            Bn[s2][1][i] = (__bf16)(ds[jj] * prev[1][jj]);
                            Bn[s2][2][i] = (__bf16)(ds[jj] * prev[2][jj]);
                            Bn[s2][3][i] = (__bf16)(ds[jj] * prev[3][jj]);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) prev[q] = acc[q];
                    __builtin_amdgcn_sched_barrier(0);
                }
                mlp_store<NT, kHalf, kHalf>(pf, nbuf);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int q = 0; q < 4; ++q) B[s][q] = Bn[s][q];
            } else {
                mlp_fetch<NT, 0, kPer>(m, next, pf);
                // output layer: one 16-row tile (rows >= 6 zero)
                floatx4 o[4] = {floatx4{}, floatx4{}, floatx4{}, floatx4{}};
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(Wl + 32 * s);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        o[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, B[s][q], o[q], 0, 0, 0);
                }
                // lane (g, col) holds outputs 4g + jj of particle 16p + col: into its slot in LDS
                if (g < 2) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj)
                            if (4 * g + jj < kMlpOut)
                                yw[(16 * p + col) * (4 * kMlpOut) + q * kMlpOut + 4 * g + jj] = o[q][jj] * kMlpLn2;
                }
                mlp_store<NT, 0, kPer>(pf, nbuf);
            }
            cur ^= 1;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float *mine = yw + l * (4 * kMlpOut);
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) {
        y[o] = mine[o] + L.co[o];
        dy[0][o] = mine[kMlpOut + o];
        dy[1][o] = mine[2 * kMlpOut + o];
        dy[2][o] = mine[3 * kMlpOut + o];
    }
}

// x^p for the envelope: small whole exponents (the usual r^-1 and r^-2 falls)
// by multiplication, others by pow.  The exponent is the same for every lane.
template <typename R>
__device__ __forceinline__ R env_pow(R x, R p) {
    if (p == (R)1) return x;
    if (p == (R)2) return x * x;
    if (p == (R)3) return x * x * x;
    if (p == (R)0) return (R)1;
    return pow(x, p);
}

// Field components (B, E, grad|B|, (b.grad)b in the local basis) from the
// network outputs at (r, th): envelope S_c (r_ref/r)^p_c, derivative chain rule,
// metric factors and connection terms.  Returns false for a non-finite result.
template <typename R>
__device__ __forceinline__ bool mlp_assemble(const MlpArgs &m, R r, R th, const float y[kMlpOut],
                                             const float dy[3][kMlpOut], R g[12]) {
    R env[kMlpOut], denv[kMlpOut];
#pragma unroll
    for (int c = 0; c < kMlpOut; ++c) {
        env[c] = (R)m.scale[c] * env_pow((R)m.r_ref / r, (R)m.power[c]);
        denv[c] = -(R)m.power[c] * env[c] / r;
    }
    R B[3], dB[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        B[i] = env[i] * (R)y[i];
        g[3 + i] = env[3 + i] * (R)y[3 + i];
        dB[0][i] = denv[i] * (R)y[i] + env[i] * (R)dy[0][i];
        dB[1][i] = env[i] * (R)dy[1][i];
        dB[2][i] = env[i] * (R)dy[2][i];
    }
    const R Bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    const R b[3] = {B[0] / Bm, B[1] / Bm, B[2] / Bm};
    R dBm[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) dBm[d] = dB[d][0] * b[0] + dB[d][1] * b[1] + dB[d][2] * b[2];
    const R st = sin(th), ct = cos(th);
    const R ir = (R)1 / r, irs = ir / st, cot = ct / st;
    g[0] = B[0]; g[1] = B[1]; g[2] = B[2];
    g[6] = dBm[0];
    g[7] = dBm[1] * ir;
    g[8] = dBm[2] * irs;
    R D[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const R db0 = (dB[0][i] - b[i] * dBm[0]) / Bm;
        const R db1 = (dB[1][i] - b[i] * dBm[1]) / Bm;
        const R db2 = (dB[2][i] - b[i] * dBm[2]) / Bm;
        D[i] = b[0] * db0 + b[1] * ir * db1 + b[2] * irs * db2;
    }
    g[9] = D[0] - (b[1] * b[1] + b[2] * b[2]) * ir;
    g[10] = D[1] + b[0] * b[1] * ir - b[2] * b[2] * cot * ir;
    g[11] = D[2] + b[0] * b[2] * ir + b[1] * b[2] * cot * ir;
    R sum = 0;
#pragma unroll
    for (int c = 0; c < 12; ++c) sum += g[c];
    return isfinite(sum);
}

}  // namespace gc
