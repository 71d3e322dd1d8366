// mlp.hip -- the schedule-predicting network on gfx950: 32 -> 64 -> 64 -> 12,
// ReLU, softmax cross-entropy, Adam (Kingma & Ba 2015), all fp32.
//
// The network is tiny (7,052 parameters, ~14 kFLOP per sample): the forward,
// input-gradient, loss and Adam kernels give one thread one output element,
// the weight-gradient kernel one workgroup one output unit; every sum runs in
// a fixed order, so the results are deterministic run to run.  Parameter layout (flat, row-major):
// W1[64,32] b1[64] W2[64,64] b2[64] W3[12,64] b3[12].
//
#include "internal.h"
#include "mlp.h"

namespace hicr {

// Y[b,o] = bias[o] + sum_i W[o,i] X[b,i], summed from the bias in ascending
// i (the host inference uses the same order); Yact gets the ReLU.  A
// workgroup takes 256 / O samples and stages W transposed (rows padded to
// O + 1, so neither the staging stores nor the loop's reads conflict in LDS)
// and its samples' inputs: lanes then read consecutive W^T entries, where
// reading row-major W directly was a stride-I access in every lane.
constexpr int kFwdWords = kMlpHidden * (kMlpHidden + 1);
constexpr int kFwdInputs = 2048;
static_assert(kMlpIn * (kMlpHidden + 1) <= kFwdWords && kMlpHidden * (kMlpOut + 1) <= kFwdWords,
              "every layer's W^T fits the LDS stage");
static_assert((256 / kMlpHidden) * kMlpHidden <= kFwdInputs &&
                  (256 / kMlpOut) * kMlpHidden <= kFwdInputs,
              "every layer's sample inputs fit the LDS stage");
__global__ __launch_bounds__(256) void dense_fwd_kernel(const float *X, const float *W,
                                                        const float *bias, int I, int O, int B,
                                                        float *Ypre, float *Yact) {
  __shared__ float wt[kFwdWords];
  __shared__ float xs[kFwdInputs];
  const int t = threadIdx.x, S = 256 / O, P = O + 1;
  const int b0 = blockIdx.x * S;
  const int nS = B - b0 < S ? B - b0 : S;
  for (int k = t; k < I * O; k += 256) wt[(k % I) * P + k / I] = W[k];
  for (int k = t; k < nS * I; k += 256) xs[k] = X[b0 * I + k];
  __syncthreads();
  const int sm = t / O, o = t % O;
  if (sm >= nS) return;
  float acc = bias[o];
#pragma unroll 8
  for (int i = 0; i < I; i++) acc = fmaf(wt[i * P + o], xs[sm * I + i], acc);
  const int y = (b0 + sm) * O + o;
  Ypre[y] = acc;
  if (Yact) Yact[y] = acc > 0.f ? acc : 0.f;
}

// Per sample: softmax of the logits, dZ = (p - onehot(y)) / B, and the
// sample's cross-entropy log-sum-exp(z) - z_y.
__global__ __launch_bounds__(256) void softmax_xent_kernel(const float *Z, const int32_t *y,
                                                           int B, float *dZ, float *loss) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  const float *z = Z + b * kMlpOut;
  float m = z[0];
  for (int c = 1; c < kMlpOut; c++) m = fmaxf(m, z[c]);
  float sum = 0.f;
  for (int c = 0; c < kMlpOut; c++) sum += expf(z[c] - m);
  // A label outside [0, kMlpOut) is never used as an index: the sample's loss
  // is NaN (so a mean over the batch shows it) and it adds no gradient.
  const int yb = y[b];
  const bool valid = yb >= 0 && yb < kMlpOut;
  for (int c = 0; c < kMlpOut; c++) {
    const float p = expf(z[c] - m) / sum;
    dZ[b * kMlpOut + c] = valid ? (p - (c == yb ? 1.f : 0.f)) / (float)B : 0.f;
  }
  if (loss) loss[b] = valid ? (m + logf(sum)) - z[yb] : __builtin_nanf("");
}

// dX[b,i] = (sum_o dY[b,o] W[o,i]) * [Xpre[b,i] > 0]
__global__ __launch_bounds__(256) void dense_bwd_input_kernel(const float *dY, const float *W,
                                                              const float *Xpre, int I, int O,
                                                              int B, float *dX) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= B * I) return;
  const int b = t / I, i = t % I;
  float acc = 0.f;
#pragma unroll 16
  for (int o = 0; o < O; o++) acc = fmaf(dY[b * O + o], W[o * I + i], acc);
  dX[t] = Xpre[t] > 0.f ? acc : 0.f;
}

// dW[o,i] = sum_b dY[b,o] X[b,i] and db[o] = sum_b dY[b,o], one workgroup
// per output o (I <= 256).  256 / I threads share column i, each summing
// every (256 / I)-th row, so a wavefront reads consecutive columns of a row
// and every thread keeps many independent loads in flight (one thread per
// weight walking all B rows left the kernel latency-bound on a few
// workgroups).  Partial sums meet in LDS in a fixed order: the result does
// not depend on timing.
__global__ __launch_bounds__(256) void dense_bwd_weight_kernel(const float *dY, const float *X,
                                                               int I, int O, int B, float *dW,
                                                               float *db) {
  __shared__ float part[256];
  __shared__ float wsum[4];
  const int o = blockIdx.x, t = threadIdx.x;
  const int parts = 256 / I, i = t % I, p = t / I;
  float acc = 0.f;
  if (p < parts) {
#pragma unroll 16
    for (int b = p; b < B; b += parts) acc = fmaf(dY[b * O + o], X[b * I + i], acc);
  }
  part[t] = acc;
  float bs = 0.f;
  for (int b = t; b < B; b += 256) bs += dY[b * O + o];
  for (int off = 32; off > 0; off >>= 1) bs += __shfl_down(bs, off, 64);
  if ((t & 63) == 0) wsum[t >> 6] = bs;
  __syncthreads();
  if (t < I) {
    float sum = 0.f;
    for (int q = 0; q < parts; q++) sum += part[q * I + t];
    dW[o * I + t] = sum;
  }
  if (t == 0) db[o] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

__global__ __launch_bounds__(256) void mean_kernel(const float *v, int n, float *out) {
  __shared__ float part[256];
  float acc = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) acc += v[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < 256; i++) s += part[i];
    *out = s / (float)n;
  }
}

__global__ __launch_bounds__(256) void adam_kernel(float *p, const float *g, float *m, float *v,
                                                   int n, float lr, float b1, float b2, float eps,
                                                   float bc1, float bc2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

static_assert(kMlpIn <= 256 && kMlpHidden <= 256, "dense_bwd_weight_kernel spreads I columns over 256 threads");

static inline unsigned blocks(int n) { return (unsigned)((n + 255) / 256); }
// workgroups of dense_fwd_kernel: 256 / O samples each
static inline unsigned fwd_blocks(int B, int O) { return (unsigned)((B + 256 / O - 1) / (256 / O)); }

hipError_t mlp_forward(const MlpBufs &m, const float *params, const float *X, int B,
                       hipStream_t s) {
  const float *W1 = params, *b1 = W1 + kMlpHidden * kMlpIn, *W2 = b1 + kMlpHidden,
              *b2 = W2 + kMlpHidden * kMlpHidden, *W3 = b2 + kMlpHidden,
              *b3 = W3 + kMlpOut * kMlpHidden;
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(fwd_blocks(B, kMlpHidden)), dim3(256), 0, s, X, W1, b1,
                     kMlpIn, kMlpHidden, B, m.a1, m.h1);
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(fwd_blocks(B, kMlpHidden)), dim3(256), 0, s, m.h1, W2,
                     b2, kMlpHidden, kMlpHidden, B, m.a2, m.h2);
  hipLaunchKernelGGL(dense_fwd_kernel, dim3(fwd_blocks(B, kMlpOut)), dim3(256), 0, s, m.h2, W3, b3,
                     kMlpHidden, kMlpOut, B, m.z, (float *)nullptr);
  return hipGetLastError();
}

hipError_t mlp_backward(const MlpBufs &m, const float *params, const float *X, const int32_t *y,
                        int B, float *grad, float *loss_mean, hipStream_t s) {
  const float *W2 = params + kMlpHidden * kMlpIn + kMlpHidden;
  const float *W3 = W2 + kMlpHidden * kMlpHidden + kMlpHidden;
  float *gW1 = grad, *gb1 = gW1 + kMlpHidden * kMlpIn, *gW2 = gb1 + kMlpHidden,
        *gb2 = gW2 + kMlpHidden * kMlpHidden, *gW3 = gb2 + kMlpHidden,
        *gb3 = gW3 + kMlpOut * kMlpHidden;
  hipLaunchKernelGGL(softmax_xent_kernel, dim3(blocks(B)), dim3(256), 0, s, m.z, y, B, m.dz,
                     m.loss);
  hipLaunchKernelGGL(dense_bwd_weight_kernel, dim3(kMlpOut), dim3(256),
                     0, s, m.dz, m.h2, kMlpHidden, kMlpOut, B, gW3, gb3);
  hipLaunchKernelGGL(dense_bwd_input_kernel, dim3(blocks(B * kMlpHidden)), dim3(256), 0, s, m.dz,
                     W3, m.a2, kMlpHidden, kMlpOut, B, m.d2);
  hipLaunchKernelGGL(dense_bwd_weight_kernel, dim3(kMlpHidden), dim3(256), 0, s, m.d2, m.h1,
                     kMlpHidden, kMlpHidden, B, gW2, gb2);
  hipLaunchKernelGGL(dense_bwd_input_kernel, dim3(blocks(B * kMlpHidden)), dim3(256), 0, s, m.d2,
                     W2, m.a1, kMlpHidden, kMlpHidden, B, m.d1);
  hipLaunchKernelGGL(dense_bwd_weight_kernel, dim3(kMlpHidden), dim3(256),
                     0, s, m.d1, X, kMlpIn, kMlpHidden, B, gW1, gb1);
  if (loss_mean) hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, s, m.loss, B, loss_mean);
  return hipGetLastError();
}

hipError_t mlp_adam(float *p, const float *g, float *mo, float *ve, float lr, int t,
                    hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.f - powf(b1, (float)t), bc2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks(kMlpParams)), dim3(256), 0, s, p, g, mo, ve,
                     kMlpParams, lr, b1, b2, 1e-8f, bc1, bc2);
  return hipGetLastError();
}

}  // namespace hicr
