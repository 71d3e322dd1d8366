// net_fma.cpp -- the host forward pass of the schedule network, compiled
// with the host's FMA instructions (a per-file host flag): std::fmaf becomes
// one instruction instead of a library call, and the axpy loops vectorise.
// Same results as the portable build, since fmaf is exact either way.
#include "net_host.h"

namespace hicr {

uint32_t net_class_fma(const float *T, const float *x) { return net_class_axpy(T, x); }

}  // namespace hicr
