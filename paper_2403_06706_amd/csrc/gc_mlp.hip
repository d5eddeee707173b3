// gc_mlp.hip -- neural field: training (forward, loss, backward, Adam) with
// BF16 MFMA matrix products and FP32 accumulation/master weights; point
// evaluation of the neural field and of the trilinear grid (its judge).
#include <hip/hip_runtime.h>

#include "gc_device.h"
#include "gc_launch.h"
#include "gc_mlp.h"
#include "gc_mlp_launch.h"

namespace gc {

// ---------------------------------------------------------------------------
// Features of training rows (no tangents): H0[row][128] bf16.
// pts: SoA r[n], th[n], ph[n].
// ---------------------------------------------------------------------------
__global__ void k_mlp_features(MlpArgs m, const double *pts, int n, __bf16 *H0) {
    const int row = blockIdx.x * blockDim.y + threadIdx.y;   // blockDim = (64, 4): 64 lanes share a row
    if (row >= n) return;
    const int j = threadIdx.x;                               // phase index
    const float rt = (float)((pts[row] - (double)m.r_min) * (double)m.inv_rspan);
    const float tt = (float)(pts[n + row] * 0.3183098861837907);
    const float ph = (float)pts[2 * n + row];
    const float psi = 6.283185307179586f * (m.fa[j] * rt + m.fb[j] * tt) + m.fn[j] * ph;
    float sn, cs;
    __sincosf(psi, &sn, &cs);
    H0[(size_t)row * kMlpWidth + 2 * j] = (__bf16)sn;
    H0[(size_t)row * kMlpWidth + 2 * j + 1] = (__bf16)cs;
}

// ---------------------------------------------------------------------------
// C[row][n] = sum_k A[row][k] Bt[n][k] for 32 rows per wavefront, NT 32-wide
// column tiles.  MODE 0 (forward hidden layer): Z = C + bias, store Z (fp32)
// and silu(Z) (bf16).  MODE 1 (backward data): store C (fp32).  MODE 2
// (output layer): store C + bias for the first kMlpOut columns (fp32, n x 6).
// ---------------------------------------------------------------------------
template <int MODE, int NT>
__global__ __launch_bounds__(256) void k_mlp_gemm(const __bf16 *A, const __bf16 *Bt, const float *bias, int rows,
                                                  float *Cout, __bf16 *Hout) {
    const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = l >> 5, mrow = l & 31;
    const int row0 = (blockIdx.x * 4 + wave) * 32;
    if (row0 >= rows) return;                                   // whole wavefront idle
    floatx16 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = floatx16{};
    const int arow = row0 + mrow;
    for (int s = 0; s < 8; ++s) {
        bf16x8 a = {};
        if (arow < rows) a = *reinterpret_cast<const bf16x8 *>(A + (size_t)arow * kMlpWidth + 16 * s + 8 * half);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(Bt + (size_t)(32 * nt + mrow) * kMlpWidth + 16 * s + 8 * half);
            acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[nt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int n = 32 * nt + mrow;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = row0 + (j / 4) * 8 + half * 4 + (j % 4);
            if (row >= rows) continue;
            if (MODE == 0) {
                const float z = acc[nt][j] + bias[n];
                Cout[(size_t)row * kMlpWidth + n] = z;
                Hout[(size_t)row * kMlpWidth + n] = (__bf16)silu_f(z);
            } else if (MODE == 1) {
                Cout[(size_t)row * kMlpWidth + n] = acc[nt][j];
            } else if (n < kMlpOut) {
                Cout[(size_t)row * kMlpOut + n] = acc[nt][j] + bias[n];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient, split over row chunks: P[g][n][k] = sum_{rows of chunk g} D[r][n] H[r][k].
// Each workgroup stages 16 rows of D and H transposed in LDS, so that the
// MFMA operands (8 consecutive rows of one column) are 16-byte LDS reads.
// ---------------------------------------------------------------------------
constexpr int kWgRow = 16 + 8;   // padded LDS row (bf16) of the transposed tiles

__global__ __launch_bounds__(256) void k_mlp_wgrad(const __bf16 *D, const __bf16 *H, int rows, int chunk,
                                                   float *partial) {
    __shared__ __bf16 Dt[kMlpWidth * kWgRow];
    __shared__ __bf16 Ht[kMlpWidth * kWgRow];
    const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = l >> 5, mrow = l & 31;
    const int r_begin = blockIdx.x * chunk, r_end = min(rows, r_begin + chunk);
    floatx16 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx16{};
    for (int r0 = r_begin; r0 < r_end; r0 += 16) {
        // stage 16 x 128 of D and H, transposed: Xt[col][row]
        for (int e = threadIdx.x; e < 16 * kMlpWidth; e += 256) {
            const int rr = e / kMlpWidth, cc = e % kMlpWidth;
            const int r = r0 + rr;
            const __bf16 zero = (__bf16)0.0f;
            Dt[cc * kWgRow + rr] = r < r_end ? D[(size_t)r * kMlpWidth + cc] : zero;
            Ht[cc * kWgRow + rr] = r < r_end ? H[(size_t)r * kMlpWidth + cc] : zero;
        }
        __syncthreads();
        // A[m = n-unit][k = row] = D[row][32 wave + m];  B[k = row][n = k-unit] = H[row][32 nt + n]
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(Dt + (32 * wave + mrow) * kWgRow + 8 * half);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(Ht + (32 * nt + mrow) * kWgRow + 8 * half);
            acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[nt], 0, 0, 0);
        }
        __syncthreads();
    }
    float *P = partial + (size_t)blockIdx.x * kMlpWidth * kMlpWidth;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int nrow = 32 * wave + (j / 4) * 8 + half * 4 + (j % 4);
            P[nrow * kMlpWidth + 32 * nt + mrow] = acc[nt][j];
        }
}

// out[i] (+)= sum_g partial[g][i], i < count (deterministic order; four
// independent partial sums keep several loads in flight)
__global__ void k_sum_partials(const float *partial, int groups, int count, float *out, int accumulate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int g = 0;
    for (; g + 4 <= groups; g += 4)
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] += partial[(size_t)(g + u) * count + i];
    for (; g < groups; ++g) s[0] += partial[(size_t)g * count + i];
    const float t = (s[0] + s[1]) + (s[2] + s[3]);
    out[i] = accumulate ? out[i] + t : t;
}

// ---------------------------------------------------------------------------
// Loss of the normalized outputs at paired points (rows 0..N-1 and N..2N-1)
// and its gradient with respect to the outputs.  Per-block partial sums.
// ---------------------------------------------------------------------------
__global__ void k_mlp_loss(MlpArgs m, const double *pts, const double *tgt, const float *Y, int npair, MlpLoss L,
                           float *dY, double *loss_partial) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npair; i += gridDim.x * blockDim.x) {
        const double r1 = pts[i], r2 = pts[npair + i];
        for (int c = 0; c < kMlpOut; ++c) {
            const double e1 = (double)m.scale[c] * pow((double)m.r_ref / r1, (double)m.power[c]);
            const double e2 = (double)m.scale[c] * pow((double)m.r_ref / r2, (double)m.power[c]);
            const double t1 = tgt[(size_t)i * kMlpOut + c] / e1, t2 = tgt[(size_t)(npair + i) * kMlpOut + c] / e2;
            const double y1 = Y[(size_t)i * kMlpOut + c], y2 = Y[(size_t)(npair + i) * kMlpOut + c];
            const double d1 = y1 - t1, d12 = (y2 - y1) - (t2 - t1);
            acc += L.wc[c] * (d1 * d1 + L.beta * d12 * d12);
            dY[(size_t)i * kMlpOut + c] = (float)((2.0 * L.wc[c] * d1 - 2.0 * L.beta * L.wc[c] * d12) / npair);
            dY[(size_t)(npair + i) * kMlpOut + c] = (float)(2.0 * L.beta * L.wc[c] * d12 / npair);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_partial[blockIdx.x] = red[0] / npair;
}

// dH6 = dY Wo  (the output layer has K = 6: plain FP32; silu' is applied by k_mlp_dz)
__global__ void k_mlp_out_back(const float *dY, const float *Wo_master, int rows, float *dH) {
    const int k = threadIdx.x, row = blockIdx.x;
    if (row >= rows) return;
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kMlpOut; ++c) s += dY[(size_t)row * kMlpOut + c] * Wo_master[c * kMlpWidth + k];
    dH[(size_t)row * kMlpWidth + k] = s;
}

// Row-parallel column work: a 256-thread block takes kColRows = 64 rows, thread
// (half = tid / 128, k = tid % 128) the rows r0 + half + 2i of column k.

// dZ = dH * silu'(Z) -> bf16, and per-block column sums (bias gradient)
__global__ __launch_bounds__(256) void k_mlp_dz(const float *dH, const float *Z, int rows, __bf16 *dZ,
                                                float *bias_partial) {
    __shared__ float red[kMlpWidth];
    const int k = threadIdx.x & (kMlpWidth - 1), half = threadIdx.x >> 7;
    const int r0 = blockIdx.x * kColRows;
    float s = 0.0f;
    for (int i = half; i < kColRows; i += 2) {
        const int r = r0 + i;
        if (r >= rows) break;
        const float v = dH[(size_t)r * kMlpWidth + k] * dsilu_f(Z[(size_t)r * kMlpWidth + k]);
        dZ[(size_t)r * kMlpWidth + k] = (__bf16)v;
        s += v;
    }
    if (half) red[k] = s;
    __syncthreads();
    if (!half) bias_partial[(size_t)blockIdx.x * kMlpWidth + k] = s + red[k];
}

// output layer: dWo[c][k] = sum_r dY[r][c] H6[r][k], dco[c] = sum_r dY[r][c]  (per-block partials)
__global__ __launch_bounds__(256) void k_mlp_out_grad(const float *dY, const __bf16 *H6, int rows, float *partial) {
    __shared__ float red[kMlpOut * kMlpWidth + kMlpOut];
    const int k = threadIdx.x & (kMlpWidth - 1), half = threadIdx.x >> 7;
    const int r0 = blockIdx.x * kColRows;
    float s[kMlpOut] = {0, 0, 0, 0, 0, 0}, sb[kMlpOut] = {0, 0, 0, 0, 0, 0};
    for (int i = half; i < kColRows; i += 2) {
        const int r = r0 + i;
        if (r >= rows) break;
        const float h = (float)H6[(size_t)r * kMlpWidth + k];
#pragma unroll
        for (int c = 0; c < kMlpOut; ++c) {
            const float d = dY[(size_t)r * kMlpOut + c];
            s[c] += d * h;
            sb[c] += d;
        }
    }
    if (half) {
#pragma unroll
        for (int c = 0; c < kMlpOut; ++c) red[c * kMlpWidth + k] = s[c];
        if (k < kMlpOut) red[kMlpOut * kMlpWidth + k] = sb[k];
    }
    __syncthreads();
    if (!half) {
        float *P = partial + (size_t)blockIdx.x * (kMlpOut * kMlpWidth + kMlpOut);
#pragma unroll
        for (int c = 0; c < kMlpOut; ++c) P[c * kMlpWidth + k] = s[c] + red[c * kMlpWidth + k];
        if (k < kMlpOut) P[kMlpOut * kMlpWidth + k] = sb[k] + red[kMlpOut * kMlpWidth + k];
    }
}

// ---------------------------------------------------------------------------
// Adam on the fp32 master parameters, then the bf16 copies used by the MFMA
// products (W row-major, W transposed, Wo).
// ---------------------------------------------------------------------------
__global__ void k_adam(float *p, float *mo, float *ve, const float *g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * mo[i] + (1.0f - b1) * gi;
    const float vi = b2 * ve[i] + (1.0f - b2) * gi * gi;
    mo[i] = mi;
    ve[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// W, WT, Wo: natural order (training products); We, Woe: evaluation order
// (columns of layers 2..6 and of the output layer permuted by mlp_perm).
__global__ void k_mlp_refresh(const float *p, __bf16 *W, __bf16 *WT, __bf16 *Wo, __bf16 *We, __bf16 *Woe) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMlpDepth * kMlpWidth * kMlpWidth) {
        const int layer = i / (kMlpWidth * kMlpWidth), e = i % (kMlpWidth * kMlpWidth);
        const int n = e / kMlpWidth, k = e % kMlpWidth;
        const __bf16 v = (__bf16)p[kMlpOffW + i];
        W[i] = v;
        WT[(size_t)layer * kMlpWidth * kMlpWidth + k * kMlpWidth + n] = v;
        const int ks = layer == 0 ? k : (k & ~31) + mlp_perm(k & 31);
        We[i] = (__bf16)p[kMlpOffW + (size_t)layer * kMlpWidth * kMlpWidth + n * kMlpWidth + ks];
    }
    if (i < kMlpOutPad * kMlpWidth) Wo[i] = (__bf16)p[kMlpOffWo + i];
    if (i < kMlpEvalRows * kMlpWidth) {
        const int n = i / kMlpWidth, k = i % kMlpWidth;
        Woe[i] = n < kMlpOut ? (__bf16)p[kMlpOffWo + n * kMlpWidth + (k & ~31) + mlp_perm(k & 31)] : (__bf16)0.0f;
    }
}

// ---------------------------------------------------------------------------
// Point evaluation: neural field (64 points per wavefront) and trilinear grid.
// pts SoA: r[n], th[n], ph[n]; out: [n][12].
// ---------------------------------------------------------------------------
constexpr int kEvalThreads = 512;   // 8 wavefronts (2 per SIMD) share the staged weights

__global__ __launch_bounds__(kEvalThreads) __attribute__((amdgpu_waves_per_eu(2)))
void k_mlp_eval(MlpArgs m, const double *pts, int n, double *out) {
    __shared__ MlpLds<kEvalThreads> L;
    mlp_lds_init(m, L);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int ii = i < n ? i : n - 1;                 // idle lanes evaluate a valid point
    const double r = pts[ii], th = pts[n + ii], ph = pts[2 * n + ii];
    float y[kMlpOut], dy[3][kMlpOut];
    mlp_block<kEvalThreads>(m, (float)r, (float)th, (float)ph, L, y, dy);
    double g[12];
    const bool ok = mlp_assemble<double>(m, r, th, y, dy, g);
    if (i < n)
        for (int c = 0; c < 12; ++c) out[(size_t)i * 12 + c] = ok ? g[c] : __builtin_nan("");
}

template <int FDT>
__global__ void k_field_sample(FieldDev f, const double *pts, int n, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double g[12];
    const bool ok = gather<FDT, double>(f, pts[i], pts[n + i], pts[2 * n + i], g);
    for (int c = 0; c < 12; ++c) out[(size_t)i * 12 + c] = ok ? g[c] : __builtin_nan("");
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t mlp_launch_features(const MlpArgs &m, const double *pts, int n, __bf16 *H0, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_features, dim3((n + 3) / 4), dim3(64, 4), 0, s, m, pts, n, H0);
    return hipGetLastError();
}

hipError_t mlp_launch_forward_layer(const __bf16 *A, const __bf16 *W, const float *bias, int rows, float *Z,
                                    __bf16 *H, hipStream_t s) {
    hipLaunchKernelGGL((k_mlp_gemm<0, 4>), dim3((rows + 127) / 128), dim3(256), 0, s, A, W, bias, rows, Z, H);
    return hipGetLastError();
}

hipError_t mlp_launch_output(const __bf16 *A, const __bf16 *Wo, const float *co, int rows, float *Y, hipStream_t s) {
    hipLaunchKernelGGL((k_mlp_gemm<2, 1>), dim3((rows + 127) / 128), dim3(256), 0, s, A, Wo, co, rows, Y,
                       (__bf16 *)nullptr);
    return hipGetLastError();
}

hipError_t mlp_launch_backward_data(const __bf16 *dZ, const __bf16 *WT, int rows, float *dH, hipStream_t s) {
    hipLaunchKernelGGL((k_mlp_gemm<1, 4>), dim3((rows + 127) / 128), dim3(256), 0, s, dZ, WT, (const float *)nullptr,
                       rows, dH, (__bf16 *)nullptr);
    return hipGetLastError();
}

hipError_t mlp_launch_wgrad(const __bf16 *D, const __bf16 *H, int rows, int groups, float *partial, float *out,
                            hipStream_t s) {
    const int chunk = ((rows + groups - 1) / groups + 15) / 16 * 16;
    const int g = (rows + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(g), dim3(256), 0, s, D, H, rows, chunk, partial);
    const int count = kMlpWidth * kMlpWidth;
    hipLaunchKernelGGL(k_sum_partials, dim3((count + 255) / 256), dim3(256), 0, s, partial, g, count, out, 0);
    return hipGetLastError();
}

hipError_t mlp_launch_loss(const MlpArgs &m, const double *pts, const double *tgt, const float *Y, int npair,
                           const MlpLoss &L, float *dY, double *loss_partial, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_loss, dim3(blocks), dim3(256), 0, s, m, pts, tgt, Y, npair, L, dY, loss_partial);
    return hipGetLastError();
}

hipError_t mlp_launch_out_back(const float *dY, const float *Wo_master, int rows, float *dH, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_out_back, dim3(rows), dim3(kMlpWidth), 0, s, dY, Wo_master, rows, dH);
    return hipGetLastError();
}

hipError_t mlp_launch_dz(const float *dH, const float *Z, int rows, __bf16 *dZ, float *bias_partial,
                         float *bias_out, hipStream_t s) {
    const int g = (rows + kColRows - 1) / kColRows;
    hipLaunchKernelGGL(k_mlp_dz, dim3(g), dim3(256), 0, s, dH, Z, rows, dZ, bias_partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kMlpWidth), 0, s, bias_partial, g, kMlpWidth, bias_out, 0);
    return hipGetLastError();
}

hipError_t mlp_launch_out_grad(const float *dY, const __bf16 *H6, int rows, float *partial, float *dWo, float *dco,
                               hipStream_t s) {
    const int g = (rows + kColRows - 1) / kColRows;
    hipLaunchKernelGGL(k_mlp_out_grad, dim3(g), dim3(256), 0, s, dY, H6, rows, partial);
    const int count = kMlpOut * kMlpWidth + kMlpOut;
    // the partial block is [c][k] then [c]: sum into a staging area laid out the same way
    hipLaunchKernelGGL(k_sum_partials, dim3((count + 255) / 256), dim3(256), 0, s, partial, g, count,
                       partial + (size_t)g * count, 0);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(dWo, partial + (size_t)g * count, kMlpOut * kMlpWidth * sizeof(float),
                           hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dco, partial + (size_t)g * count + kMlpOut * kMlpWidth, kMlpOut * sizeof(float),
                           hipMemcpyDeviceToDevice, s);
    return e;
}


hipError_t mlp_launch_adam(float *p, float *mo, float *ve, const float *g, int n, float lr, float b1, float b2,
                           float eps, int step, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, mo, ve, g, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_launch_refresh(const float *p, __bf16 *W, __bf16 *WT, __bf16 *Wo, __bf16 *We, __bf16 *Woe,
                              hipStream_t s) {
    const int n = kMlpDepth * kMlpWidth * kMlpWidth;
    hipLaunchKernelGGL(k_mlp_refresh, dim3((n + 255) / 256), dim3(256), 0, s, p, W, WT, Wo, We, Woe);
    return hipGetLastError();
}

hipError_t mlp_launch_eval(const MlpArgs &m, const double *pts, int n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_eval, dim3((n + kEvalThreads - 1) / kEvalThreads), dim3(kEvalThreads), 0, s, m, pts, n,
                       out);
    return hipGetLastError();
}

hipError_t launch_field_sample(const FieldDev &f, const double *pts, int n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 grid((n + 255) / 256), block(256);
    switch (f.dtype) {
        case GC_F64: hipLaunchKernelGGL(k_field_sample<GC_F64>, grid, block, 0, s, f, pts, n, out); break;
        case GC_F32: hipLaunchKernelGGL(k_field_sample<GC_F32>, grid, block, 0, s, f, pts, n, out); break;
        default:     hipLaunchKernelGGL(k_field_sample<GC_F16>, grid, block, 0, s, f, pts, n, out); break;
    }
    return hipGetLastError();
}

}  // namespace gc
