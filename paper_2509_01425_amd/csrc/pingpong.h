// pingpong.h -- arguments of the two-endpoint ping-pong kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hicr {

struct PingPongArgs {
  uint64_t src, dst, ring_a, ring_b, buf;  // 16-byte aligned device addresses
  uint64_t size;                            // message bytes
  uint32_t W;                               // workgroups per endpoint
  uint32_t reps;                            // round trips
  uint64_t *ctr;      // [4] A arrived, A freed, B arrived, B freed (stripes), zeroed
  uint64_t *t_start;  // [reps] pinger clock before each push (100 MHz)
  uint64_t *t_end;    // [reps] pinger clock after reading each echo
  uint32_t *err;      // time-out flag
  uint64_t timeout_ticks;
};

hipError_t launch_pingpong(const PingPongArgs &a, hipStream_t s);
int pingpong_occupancy(int *wgs_per_cu);

}  // namespace hicr
