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

// Everything an evaluation needs (passed by value to kernels).
struct MlpArgs {
    const __bf16 *W;      // [6][128][128] bf16, row = output unit
    const __bf16 *Wo;     // [32][128] bf16 (rows >= 6 are zero)
    const float *c;       // [6][128]
    const float *co;      // [32]
    float fa[kMlpFreq], fb[kMlpFreq], fn[kMlpFreq];   // frequencies a_j, b_j, n_j
    float r_min, inv_rspan, r_ref;
    float scale[kMlpOut], power[kMlpOut];
};

// Per-wavefront LDS: 64 rows x (128 + 8) bf16 activations + 16 x 4 x 6 outputs.
constexpr int kMlpLdsRow = kMlpWidth + 8;
constexpr int kMlpLdsWaveBytes = 64 * kMlpLdsRow * 2 + 16 * 4 * kMlpOut * 4;

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// Evaluate the network and its three tangents for the 64 particles of this
// wavefront (one per lane).  Must be called by all 64 lanes together.  Output
// per lane: y[6] and dy[d][6] = dy / d(r, th, ph)[d].
//
// Matrix-core tiling (v_mfma_f32_32x32x16_bf16): particles are taken 16 at a
// time; their 64 rows are [16 values | 16 d/dr] (row tile 0) and
// [16 d/dth | 16 d/dph] (row tile 1).  In the MFMA accumulator layout a lane
// holds the same rows of both tiles, so a value row and its three tangent rows
// meet in one lane and the activation (silu, and silu' times the tangent) is
// lane-local.  Between layers the activations go through the wavefront's LDS
// tile to reach the input-operand layout.
__device__ __forceinline__ void mlp_wave(const MlpArgs &m, float r, float th, float ph, unsigned char *lds,
                                         float y[kMlpOut], float dy[3][kMlpOut]) {
    const int l = threadIdx.x & 63;
    const int half = l >> 5, mrow = l & 31;
    __bf16 *act = reinterpret_cast<__bf16 *>(lds);
    float *yout = reinterpret_cast<float *>(lds + 64 * kMlpLdsRow * 2);
    const float two_pi = 6.283185307179586f;
    for (int q = 0; q < 4; ++q) {
        // position of the particle of this lane's rows
        const int src = 16 * q + (mrow & 15);
        const float pr = __shfl(r, src), pth = __shfl(th, src), pph = __shfl(ph, src);
        const float rt = (pr - m.r_min) * m.inv_rspan, tt = pth * 0.3183098861837907f;
        const int kind0 = mrow >> 4;           // tile 0: 0 value, 1 d/dr; tile 1: 2 d/dth, 3 d/dph
        floatx16 acc[2][4];
        // ---------------- layer 1: inputs are the Fourier features
        for (int t = 0; t < 2; ++t)
            for (int nt = 0; nt < 4; ++nt) acc[t][nt] = floatx16{};
        for (int s = 0; s < 8; ++s) {
            bf16x8 a0, a1;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = 8 * s + 4 * half + i;            // phase index of features 2j, 2j+1
                const float psi = two_pi * (m.fa[j] * rt + m.fb[j] * tt) + m.fn[j] * pph;
                float sn, cs;
                __sincosf(psi, &sn, &cs);
                const float dr = two_pi * m.fa[j] * m.inv_rspan, dth = 2.0f * m.fb[j], dph = m.fn[j];
                // tile 0: value (kind 0) or d/dr (kind 1); tile 1: d/dth (2) or d/dph (3)
                const float d0 = kind0 ? dr : 0.0f, d1 = kind0 ? dph : dth;
                a0[2 * i] = (__bf16)(kind0 ? cs * d0 : sn);
                a0[2 * i + 1] = (__bf16)(kind0 ? -sn * d0 : cs);
                a1[2 * i] = (__bf16)(cs * d1);
                a1[2 * i + 1] = (__bf16)(-sn * d1);
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const bf16x8 b = *reinterpret_cast<const bf16x8 *>(m.W + (size_t)(32 * nt + mrow) * kMlpWidth + 16 * s + 8 * half);
                acc[0][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b, acc[0][nt], 0, 0, 0);
                acc[1][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b, acc[1][nt], 0, 0, 0);
            }
        }
        for (int layer = 0; layer < kMlpDepth; ++layer) {
            if (layer > 0) {
                // ---------------- layers 2..6: inputs from the LDS tile
                for (int t = 0; t < 2; ++t)
                    for (int nt = 0; nt < 4; ++nt) acc[t][nt] = floatx16{};
                const __bf16 *Wl = m.W + (size_t)layer * kMlpWidth * kMlpWidth;
                for (int s = 0; s < 8; ++s) {
                    const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(act + mrow * kMlpLdsRow + 16 * s + 8 * half);
                    const bf16x8 a1 = *reinterpret_cast<const bf16x8 *>(act + (32 + mrow) * kMlpLdsRow + 16 * s + 8 * half);
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(Wl + (size_t)(32 * nt + mrow) * kMlpWidth + 16 * s + 8 * half);
                        acc[0][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b, acc[0][nt], 0, 0, 0);
                        acc[1][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b, acc[1][nt], 0, 0, 0);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            // epilogue: bias + silu on value rows, silu'(z) * tangent on tangent rows
            const float *cl = m.c + layer * kMlpWidth;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int n = 32 * nt + mrow;
                const float bias = cl[n];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int row = (j / 4) * 8 + half * 4 + (j % 4);        // value row of a particle
                    const float z = acc[0][nt][j] + bias;
                    const float ds = dsilu_f(z);
                    act[row * kMlpLdsRow + n] = (__bf16)silu_f(z);
                    act[(row + 16) * kMlpLdsRow + n] = (__bf16)(ds * acc[0][nt][j + 8]);
                    act[(32 + row) * kMlpLdsRow + n] = (__bf16)(ds * acc[1][nt][j]);
                    act[(48 + row) * kMlpLdsRow + n] = (__bf16)(ds * acc[1][nt][j + 8]);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        // ---------------- output layer (one padded 32-wide tile)
        floatx16 o0 = {}, o1 = {};
        for (int s = 0; s < 8; ++s) {
            const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(act + mrow * kMlpLdsRow + 16 * s + 8 * half);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8 *>(act + (32 + mrow) * kMlpLdsRow + 16 * s + 8 * half);
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(m.Wo + (size_t)mrow * kMlpWidth + 16 * s + 8 * half);
            o0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b, o0, 0, 0, 0);
            o1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b, o1, 0, 0, 0);
        }
        if (mrow < kMlpOut) {
            const float bias = m.co[mrow];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int p = (j / 4) * 8 + half * 4 + (j % 4);              // particle within the pass
                yout[(p * 4 + 0) * kMlpOut + mrow] = o0[j] + bias;
                yout[(p * 4 + 1) * kMlpOut + mrow] = o0[j + 8];
                yout[(p * 4 + 2) * kMlpOut + mrow] = o1[j];
                yout[(p * 4 + 3) * kMlpOut + mrow] = o1[j + 8];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if ((l >> 4) == q) {
            const int p = l & 15;
#pragma unroll
            for (int c = 0; c < kMlpOut; ++c) {
                y[c] = yout[(p * 4 + 0) * kMlpOut + c];
                dy[0][c] = yout[(p * 4 + 1) * kMlpOut + c];
                dy[1][c] = yout[(p * 4 + 2) * kMlpOut + c];
                dy[2][c] = yout[(p * 4 + 3) * kMlpOut + c];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
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
        env[c] = (R)m.scale[c] * pow((R)m.r_ref / r, (R)m.power[c]);
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
