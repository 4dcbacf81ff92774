// Internal definitions of the learned CG force (network parameters on the device,
// launch wrappers of the inference and training kernels).
#pragma once

#include "adres_internal.h"

namespace adres {

constexpr int kHidden = 64;
constexpr int kMlpParams = kHidden + kHidden + kHidden * kHidden + kHidden + kHidden + 1;   // 4353

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef int int32x8 __attribute__((ext_vector_type(8)));   // 32 FP8 values

// Device view of the network: FP32 master parameters (layout W1[H] b1[H] W2[H*H]
// (row = output unit) b2[H] W3[H] b3) and the BF16 copy of W2 used by the MFMA.
struct MlpDev {
    const float *w1, *b1, *w2, *b2, *w3;   // w3[kHidden] is b3
    const __bf16 *w2_bf16;    // W2, row = output unit
    const __bf16 *w2t_bf16;   // W2 transposed, row = input unit
    // FP8 variant: W2 / s_w in E4M3 (OCP), row-major bytes, and the scales
    // {s_w s_g, 1 / s_g, 1 / (s_w s_g)} (s_g bounds |h1| / ln 2 / 448)
    const int *w2_fp8;
    const float *fp8_scale;
    bool fp8;                 // layer 2 on FP8 matrix cores (else BF16)
    double rc, scale, tw, r_min;
};

void launch_mlp_forward_r(hipStream_t s, const MlpDev &M, const DevParams &P, const double *r, float *f, int64_t n,
                          Ctrl *ctrl);
// pairs: half-list slot pairs, their number read from n_dev (at most n_cap)
void launch_mlp_forward_pairs(hipStream_t s, const MlpDev &M, const DevParams &P, const int2 *pairs,
                              const double4 *Rw, float *f, const int *n_dev, int64_t n_cap, Ctrl *ctrl,
                              int check_halt, int step);
// FP32 master -> FP8 copy of W2 and the per-tensor scales of the FP8 variant
void launch_mlp_fp8_prepare(hipStream_t s, const float *params, int *w2_fp8, float *scale);
// FP32 master -> BF16 copies of W2 and of its transpose
void launch_mlp_convert(hipStream_t s, const float *params, __bf16 *w2_bf16, __bf16 *w2t_bf16);

// force matching
int mlp_backward_waves();
int mlp_reduce_chunks();   // partial sums of the fixed-order gradient reduction
void launch_fm_residual(hipStream_t s, int n, const int *perm, const double *F, const double *fmap, double *e,
                        double *part, int *n_part);
void launch_loss_accumulate(hipStream_t s, const double *part, int n_part, double c, double *loss);
void launch_mlp_backward(hipStream_t s, const MlpDev &M, const DevParams &P, const int2 *pairs, const int *n_dev,
                         const double4 *Rw, const double *e, double c2, float *gpart, double *gred, double *grad);
void launch_zero(hipStream_t s, double *a, int n);
void launch_adam(hipStream_t s, float *params, float *m, float *v, const double *grad, double lr, double b1,
                 double b2, double bc1, double bc2, double eps);

}  // namespace adres
