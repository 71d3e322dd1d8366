// pingpong.hip -- the ping-pong benchmark of the paper's Test Case 1 on one
// GPU: two endpoints connected by two opposing channels of one-message
// capacity.  The pinger pushes a message into channel A and waits for its
// echo on channel B; the ponger takes each message from A into its own
// buffer, frees A, and pushes the buffer into B once the pinger has freed B.
//
// Each endpoint is a group of W workgroups: message bytes are striped over
// the group (workgroup w owns stripe w), and each channel's counters count
// stripes -- a channel's tail (`arrived`) and head (`freed`) advance by W per
// message, so a message is visible once all of its stripes are, and a ring
// is free once every stripe has been read.  W = 1 is a single workgroup per
// endpoint; large messages use many so the copies run at memory speed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pingpong.h"

namespace hicr {

#define GLOBAL __attribute__((address_space(1)))
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Block copy of n bytes between 16-byte aligned addresses (n a multiple of 16
// except possibly the last stripe, whose tail is copied byte by byte).
__device__ __forceinline__ void block_copy(uint64_t d, uint64_t s, uint64_t n, uint32_t t) {
  const uint64_t nv = n >> 4;
  for (uint64_t b = 0; b < nv; b += 256 * 4) {
    v4u r[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint64_t i = b + t + 256 * k;
      if (i < nv) r[k] = *(const GLOBAL v4u *)(s + 16 * i);
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint64_t i = b + t + 256 * k;
      if (i < nv) *(GLOBAL v4u *)(d + 16 * i) = r[k];
    }
  }
  const uint64_t tail = n & 15;
  if (t < tail)
    *(GLOBAL unsigned char *)(d + 16 * nv + t) = *(const GLOBAL unsigned char *)(s + 16 * nv + t);
}

__device__ __forceinline__ bool wait_at_least(const uint64_t *ctr, uint64_t v, uint64_t deadline,
                                              uint32_t *err) {
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) {
    __builtin_amdgcn_s_sleep(1);
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (wall_clock64() > deadline) {
      __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

__global__ __launch_bounds__(256) void pingpong_kernel(PingPongArgs a) {
  __shared__ uint32_t ok;
  const uint32_t t = threadIdx.x;
  const bool pinger = blockIdx.x < a.W;
  const uint32_t w = pinger ? blockIdx.x : blockIdx.x - a.W;
  // stripe w of an s-byte message: 16-byte multiples, the last takes the rest
  const uint64_t stripe = ((a.size + a.W - 1) / a.W + 15) & ~(uint64_t)15;
  const uint64_t lo = (uint64_t)w * stripe < a.size ? (uint64_t)w * stripe : a.size;
  const uint64_t hi = lo + stripe < a.size ? lo + stripe : a.size;
  const uint64_t W = a.W;
  uint64_t deadline = wall_clock64() + a.timeout_ticks;
  // wait until *ctr >= v: thread 0 polls and acquires, and the barrier
  // orders every other wave's later accesses after that acquire (one L2
  // invalidate per workgroup, not one per wave)
  auto wait = [&](const uint64_t *ctr, uint64_t v) {
    if (t == 0) ok = wait_at_least(ctr, v, deadline, a.err);
    __syncthreads();
    return ok != 0;
  };
  // the barrier orders every wave's copies before thread 0's release, which
  // makes them visible device-wide before one stripe is counted (one L2
  // write-back per workgroup, not one per wave)
  auto signal = [&](uint64_t *ctr) {
    __syncthreads();
    if (t == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  for (uint32_t k = 0; k < a.reps; k++) {
    if (pinger) {
      if (w == 0 && t == 0) a.t_start[k] = wall_clock64();
      if (!wait(&a.ctr[1], W * k)) return;       // A is free of message k-1
      block_copy(a.ring_a + lo, a.src + lo, hi - lo, t);
      signal(&a.ctr[0]);                         // A: stripe arrived
      if (!wait(&a.ctr[2], W * (k + 1))) return; // B holds the echo
      block_copy(a.dst + lo, a.ring_b + lo, hi - lo, t);
      signal(&a.ctr[3]);                         // B: stripe freed
      if (w == 0 && t == 0) a.t_end[k] = wall_clock64();
    } else {
      if (!wait(&a.ctr[0], W * (k + 1))) return; // A holds message k
      block_copy(a.buf + lo, a.ring_a + lo, hi - lo, t);
      signal(&a.ctr[1]);                         // A: stripe freed
      if (!wait(&a.ctr[3], W * k)) return;       // B is free of message k-1
      block_copy(a.ring_b + lo, a.buf + lo, hi - lo, t);
      signal(&a.ctr[2]);                         // B: stripe arrived
    }
    deadline = wall_clock64() + a.timeout_ticks;
  }
}

hipError_t launch_pingpong(const PingPongArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(pingpong_kernel, dim3(2 * a.W), dim3(256), 0, s, a);
  return hipGetLastError();
}

int pingpong_occupancy(int *wgs_per_cu) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, pingpong_kernel, 256, 0);
}

}  // namespace hicr
