// Internal definitions of the learned CG force (network parameters on the device,
// launch wrappers of the inference and training kernels).
#pragma once

#include "adres_internal.h"

namespace adres {

constexpr int kHidden = 64;
constexpr int kMlpParams = kHidden + kHidden + kHidden * kHidden + kHidden + kHidden + 1;   // 4353

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// Device view of the network: FP32 master parameters (layout W1[H] b1[H] W2[H*H]
// (row = output unit) b2[H] W3[H] b3) and the BF16 copy of W2 used by the MFMA.
struct MlpDev {
    const float *w1, *b1, *w2, *b2, *w3;   // w3[kHidden] is b3
    const __bf16 *w2_bf16;
    double rc, scale, tw, r_min;
};

void launch_mlp_forward_r(hipStream_t s, const MlpDev &M, const DevParams &P, const double *r, float *f, int64_t n,
                          Ctrl *ctrl);
void launch_mlp_forward_pairs(hipStream_t s, const MlpDev &M, const DevParams &P, const int2 *pairs,
                              const double4 *Rw, float *f, int64_t n, Ctrl *ctrl, int check_halt, int step);
// FP32 master -> BF16 W2 copy
void launch_mlp_convert(hipStream_t s, const float *params, __bf16 *w2_bf16);

}  // namespace adres
