// mlp.h -- the schedule-predicting network (shared by host and kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace hicr {

constexpr int kMlpIn = 32, kMlpHidden = 64, kMlpOut = 12;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden +
                           kMlpHidden + kMlpOut * kMlpHidden + kMlpOut;  // 7,052
static_assert(kMlpParams == 7052, "parameter count");

// Activations and gradients of one mini-batch of B samples (device).
struct MlpBufs {
  float *a1, *h1, *a2, *h2, *z;  // pre-activations / activations / logits
  float *dz, *d2, *d1;           // gradients w.r.t. z, a2, a1
  float *loss;                   // per-sample loss
};

hipError_t mlp_forward(const MlpBufs &m, const float *params, const float *X, int B,
                       hipStream_t s);
hipError_t mlp_backward(const MlpBufs &m, const float *params, const float *X, const int32_t *y,
                        int B, float *grad, float *loss_mean, hipStream_t s);
hipError_t mlp_adam(float *p, const float *g, float *m, float *v, float lr, int t, hipStream_t s);

// Host mirror of the histogram feature: bin floor(log2 s) capped at 31,
// size 0 in bin 0; feature log2(1 + count).
void batch_features(const uint64_t *sizes, uint64_t n, size_t stride_bytes, float *out32);

}  // namespace hicr
