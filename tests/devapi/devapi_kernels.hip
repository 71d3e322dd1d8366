// devapi_kernels.hip -- test kernels for the device-side channel API
// (hicr_device.h): one producer workgroup and one consumer workgroup of the
// caller's own kernel move messages through one ring.  Test infrastructure;
// every retry loop ends at a device-clock deadline.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hicr_device.h"

namespace {

__device__ bool expired(uint64_t deadline, uint32_t *err) {
  if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
  if (wall_clock64() > deadline) {
    __hip_atomic_fetch_or(err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
  }
  return false;
}

__device__ void copy_bytes(uint64_t d, uint64_t s, uint64_t n, uint32_t t) {
  for (uint64_t i = t; i < n; i += blockDim.x) *(unsigned char *)(d + i) = *(const unsigned char *)(s + i);
}

// Workgroup 0 pushes messages m = 0..n-1 (bytes [off[m], off[m] + size[m]) of
// src); workgroup 1 takes them in order, up to `batch` per pop, and writes
// them back to back at out.  eagain[0] counts full-ring retries.
__global__ __launch_bounds__(256) void devapi_pipe(hicr_dev_ring r, uint64_t src, const uint64_t *off,
                                                   const uint64_t *size, uint64_t n, uint64_t out,
                                                   uint32_t batch, uint64_t timeout_ticks,
                                                   uint32_t *err, uint64_t *eagain) {
  __shared__ hicr_dev_span sp[8];
  __shared__ uint32_t ok, got;
  const uint32_t t = threadIdx.x;
  const uint64_t deadline = wall_clock64() + timeout_ticks;
  if (blockIdx.x == 0) {
    for (uint64_t m = 0; m < n; m++) {
      if (t == 0) {
        ok = 1;
        for (;;) {
          const int rc = hicr_dev_push_reserve(&r, size[m], &sp[0]);
          if (rc == HICR_OK) break;
          if (rc != HICR_EAGAIN) {
            __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
          eagain[0]++;
          __builtin_amdgcn_s_sleep(2);
          if (expired(deadline, err)) {
            ok = 0;
            break;
          }
        }
      }
      __syncthreads();
      if (!ok) return;
      copy_bytes(sp[0].addr0, src + off[m], sp[0].len0, t);
      copy_bytes(sp[0].addr1, src + off[m] + sp[0].len0, sp[0].len1, t);
      __syncthreads();
      if (t == 0) hicr_dev_push_commit(&r, &sp[0]);
      __syncthreads();
    }
  } else {
    uint64_t done = 0, pos = 0;
    while (done < n) {
      if (t == 0) {
        ok = 1;
        got = 0;
        for (;;) {
          while (got < batch && got < 8 && done + got < n &&
                 hicr_dev_peek(&r, got, &sp[got]) == HICR_OK)
            got++;
          if (got) break;
          __builtin_amdgcn_s_sleep(2);
          if (expired(deadline, err)) {
            ok = 0;
            break;
          }
        }
      }
      __syncthreads();
      if (!ok) return;
      for (uint32_t k = 0; k < got; k++) {
        copy_bytes(out + pos, sp[k].addr0, sp[k].len0, t);
        copy_bytes(out + pos + sp[k].len0, sp[k].addr1, sp[k].len1, t);
        pos += sp[k].bytes;
      }
      __syncthreads();
      if (t == 0 && hicr_dev_pop(&r, got) != HICR_OK)
        __hip_atomic_fetch_or(err, 4u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      done += got;
      __syncthreads();
    }
  }
}

}  // namespace

extern "C" int devapi_pipe_run(const hicr_dev_ring *r, uint64_t src, const uint64_t *off_dev,
                               const uint64_t *size_dev, uint64_t n, uint64_t out, uint32_t batch,
                               uint64_t timeout_ticks, uint32_t *err_dev, uint64_t *eagain_dev) {
  if (!r || batch < 1 || batch > 8) return -1;
  hipLaunchKernelGGL(devapi_pipe, dim3(2), dim3(256), 0, 0, *r, src, off_dev, size_dev, n, out,
                     batch, timeout_ticks, err_dev, eagain_dev);
  if (hipGetLastError() != hipSuccess) return -2;
  return hipDeviceSynchronize() == hipSuccess ? 0 : -3;
}
