// mlp.hpp -- device view of the prefilter network's state and the launch
// wrappers of its kernels (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace ej {

constexpr int MLP_HIDDEN = 256;
constexpr int MLP_OUT = 64;

// Pointers into a state block (layout fixed by the C ABI).
struct MlpDev {
    int dim = 0, Dp = 0;       // input width and its padding to 64
    int64_t np = 0;            // parameters: W1 (dim x 256), b1, W2 (256 x 64), b2
    float* P = nullptr;        // FP32 masters, flat in that order
    float* G = nullptr;        // gradients of the last step (same layout)
    float* M = nullptr;        // Adam first moments
    float* V = nullptr;        // Adam second moments
    uint16_t* W1t = nullptr;   // BF16 W1^T, 256 x Dp (zero beyond dim)
    uint16_t* W2t = nullptr;   // BF16 W2^T, 64 x 256
    int64_t* step = nullptr;   // Adam steps taken
};

struct MlpHyper {
    float lr, beta1, beta2, eps, lambda, theta_lo;
    bool grad_only;
};

// scratch of one training step of B pairs (2B rows)
struct MlpTrainWs {
    float* Xb;   // 2B x Dp gathered rows
    float* A1;   // 2B x 256 pre-activations
    float* Z;    // 2B x 64
    float* dZ;   // 2B x 64
    float* dA1;  // 2B x 256
};

hipError_t launch_mlp_init(const MlpDev& m, const float* params, hipStream_t st);
// after masters, moments and step were written into the block: zero the
// gradients and rebuild the BF16 copies
hipError_t launch_mlp_restored(const MlpDev& m, hipStream_t st);
hipError_t launch_mlp_train_step(const MlpDev& m, const uint16_t* X, int64_t ldx, int64_t rows,
                                 const int32_t* pr, const int32_t* ps, const float* t, int B,
                                 const MlpHyper& hp, const MlpTrainWs& w, float* loss,
                                 hipStream_t st);
// U (n x 64) from prepared rows X (Dp BF16 values per row, rows up to a
// multiple of 128 readable); Hb: rows_pad x 256 BF16, Z: rows_pad x 64 FP32
hipError_t launch_mlp_forward(const MlpDev& m, const uint16_t* X, int64_t n, uint16_t* Hb,
                              float* Z, float* U, hipStream_t st);

}  // namespace ej
