// gc_mlp_launch.h -- host-side launchers of the neural-field kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "gc_internal.h"
#include "gc_mlp.h"

namespace gc {

struct MlpLoss {
    double wc[kMlpOut];   // weights of the six normalized outputs
    double beta;          // weight of the paired-difference term
};

hipError_t mlp_launch_features(const MlpArgs &m, const double *pts, int n, __bf16 *H0, hipStream_t s);
hipError_t mlp_launch_forward_layer(const __bf16 *A, const __bf16 *W, const float *bias, int rows, float *Z,
                                    __bf16 *H, hipStream_t s);
hipError_t mlp_launch_output(const __bf16 *A, const __bf16 *Wo, const float *co, int rows, float *Y, hipStream_t s);
hipError_t mlp_launch_backward_data(const __bf16 *dZ, const __bf16 *WT, int rows, float *dH, hipStream_t s);
hipError_t mlp_launch_wgrad(const __bf16 *D, const __bf16 *H, int rows, int groups, float *partial, float *out,
                            hipStream_t s);
hipError_t mlp_launch_loss(const MlpArgs &m, const double *pts, const double *tgt, const float *Y, int npair,
                           const MlpLoss &L, float *dY, double *loss_partial, int blocks, hipStream_t s);
hipError_t mlp_launch_out_back(const float *dY, const float *Wo_master, int rows, float *dH, hipStream_t s);
hipError_t mlp_launch_dz(const float *dH, const float *Z, int rows, __bf16 *dZ, float *bias_partial,
                         float *bias_out, hipStream_t s);
hipError_t mlp_launch_out_grad(const float *dY, const __bf16 *H6, int rows, float *partial, float *dWo, float *dco,
                               hipStream_t s);
constexpr int kColRows = 64;     // rows per block of the row-parallel column sums
// partial blocks of the row-parallel column sums
__host__ __device__ constexpr int mlp_col_groups(int rows) { return (rows + kColRows - 1) / kColRows; }
hipError_t mlp_launch_adam(float *p, float *mo, float *ve, const float *g, int n, float lr, float b1, float b2,
                           float eps, int step, hipStream_t s);
hipError_t mlp_launch_refresh(const float *p, __bf16 *W, __bf16 *WT, __bf16 *Wo, __bf16 *We, __bf16 *Woe,
                              hipStream_t s);
hipError_t mlp_launch_eval(const MlpArgs &m, const double *pts, int n, double *out, hipStream_t s);
hipError_t launch_field_sample(const FieldDev &f, const double *pts, int n, double *out, hipStream_t s);
hipError_t launch_push_mlp(const PushArgs &a, const MlpArgs &m, int precision, hipStream_t s);

}  // namespace gc
