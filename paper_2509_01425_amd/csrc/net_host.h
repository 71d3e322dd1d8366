// net_host.h -- the schedule network's forward pass on the host (one feature
// vector per memcpy submission), shared by the portable build in sched.cpp
// and the FMA build in net_fma.cpp.
//
// The weights are kept transposed (input-major), so every layer is a run of
// axpy updates over all outputs at once, which the compiler vectorises.  Each
// output still accumulates its inputs one by one in ascending order with a
// fused multiply-add from its bias, exactly as the device forward kernel
// does, so host and device pick the same class bit for bit.
#pragma once

#include <cmath>
#include <cstdint>

#include "mlp.h"

namespace hicr {

// Transposed copy T of the parameter vector P (layout W1 b1 W2 b2 W3 b3, each
// W output-major): same layout with each W input-major.
inline void net_transpose(const float *P, float *T) {
  int off = 0;
  auto tw = [&](int out, int in) {
    for (int o = 0; o < out; o++)
      for (int i = 0; i < in; i++) T[off + i * out + o] = P[off + o * in + i];
    off += out * in;
  };
  auto tb = [&](int out) {
    for (int o = 0; o < out; o++) T[off + o] = P[off + o];
    off += out;
  };
  tw(kMlpHidden, kMlpIn);
  tb(kMlpHidden);
  tw(kMlpHidden, kMlpHidden);
  tb(kMlpHidden);
  tw(kMlpOut, kMlpHidden);
  tb(kMlpOut);
}

// Argmax class (ties to the lowest) of the network on feature x.
inline uint32_t net_class_axpy(const float *T, const float *x) {
  const float *W1 = T, *b1 = W1 + kMlpHidden * kMlpIn, *W2 = b1 + kMlpHidden,
              *b2 = W2 + kMlpHidden * kMlpHidden, *W3 = b2 + kMlpHidden,
              *b3 = W3 + kMlpOut * kMlpHidden;
  float h1[kMlpHidden], h2[kMlpHidden], z[kMlpOut];
  for (int o = 0; o < kMlpHidden; o++) h1[o] = b1[o];
  for (int i = 0; i < kMlpIn; i++)
    for (int o = 0; o < kMlpHidden; o++) h1[o] = std::fmaf(W1[i * kMlpHidden + o], x[i], h1[o]);
  for (int o = 0; o < kMlpHidden; o++) {
    h1[o] = h1[o] > 0.f ? h1[o] : 0.f;
    h2[o] = b2[o];
  }
  for (int i = 0; i < kMlpHidden; i++)
    for (int o = 0; o < kMlpHidden; o++) h2[o] = std::fmaf(W2[i * kMlpHidden + o], h1[i], h2[o]);
  for (int o = 0; o < kMlpHidden; o++) h2[o] = h2[o] > 0.f ? h2[o] : 0.f;
  for (int o = 0; o < kMlpOut; o++) z[o] = b3[o];
  for (int i = 0; i < kMlpHidden; i++)
    for (int o = 0; o < kMlpOut; o++) z[o] = std::fmaf(W3[i * kMlpOut + o], h2[i], z[o]);
  uint32_t best = 0;
  for (int o = 1; o < kMlpOut; o++)
    if (z[o] > z[best]) best = (uint32_t)o;
  return best;
}

// The same, built with the host's FMA instructions (net_fma.cpp); call only
// where the CPU has them.
uint32_t net_class_fma(const float *T, const float *x);

}  // namespace hicr
