// fill.hip -- device-side input generation for the workloads (not part of the
// data path).  wl_fill writes the SplitMix64 byte stream (Steele, Lea & Flood,
// OOPSLA 2014: state advanced by the golden gamma, variant-13 finaliser) into
// a device range; the CPU generator in workloads/content.py computes the same
// stream independently.  wl_ref_copy is a plain aligned 16-byte copy used as
// the bandwidth reference for counter calibration.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ uint64_t sm64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// base is 16-byte aligned; word w of the range is stream output first_word + w.
__global__ __launch_bounds__(256) void fill_kernel(uint64_t base, uint64_t n_words, uint64_t seed,
                                                   uint64_t first_word) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x; 2 * p < n_words; p += stride) {
    uint64_t w = 2 * p;
    if (w + 1 < n_words) {
      typedef uint64_t v2u __attribute__((ext_vector_type(2)));
      v2u v = {sm64(seed, first_word + w), sm64(seed, first_word + w + 1)};
      *(GLOBAL v2u *)(base + 8 * w) = v;
    } else {
      *(GLOBAL uint64_t *)(base + 8 * w) = sm64(seed, first_word + w);
    }
  }
}

__global__ void fill_tail_kernel(uint64_t addr, uint32_t n, uint64_t value) {
  uint32_t t = threadIdx.x;
  if (t < n) *(GLOBAL unsigned char *)(addr + t) = (unsigned char)(value >> (8 * t));
}

__global__ __launch_bounds__(256) void ref_copy_kernel(uint64_t dst, uint64_t src, uint64_t n16) {
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride)
    *(GLOBAL v4u *)(dst + 16 * i) = *(const GLOBAL v4u *)(src + 16 * i);
}

static uint64_t host_sm64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

extern "C" {

// Fill [dev, dev + n_bytes) with bytes first_index .. first_index + n_bytes of
// the stream.  dev must be 16-byte aligned and first_index a multiple of 8.
int wl_fill(void *dev, uint64_t n_bytes, uint64_t seed, uint64_t first_index, void *stream) {
  uint64_t base = (uint64_t)dev;
  if ((base & 15) || (first_index & 7)) return -1;
  hipStream_t s = (hipStream_t)stream;
  uint64_t words = n_bytes / 8, rest = n_bytes % 8;
  if (words) {
    uint64_t blocks = (words / 2 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(fill_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, base, words, seed,
                       first_index / 8);
  }
  if (rest)
    hipLaunchKernelGGL(fill_tail_kernel, dim3(1), dim3(64), 0, s, base + 8 * words,
                       (uint32_t)rest, host_sm64(seed, first_index / 8 + words));
  return hipGetLastError() == hipSuccess ? 0 : -9;
}

// Plain copy of n_bytes (a multiple of 16; both pointers 16-byte aligned).
int wl_ref_copy(void *dst, const void *src, uint64_t n_bytes, uint32_t blocks, void *stream) {
  if (((uint64_t)dst & 15) || ((uint64_t)src & 15) || (n_bytes & 15) || blocks == 0) return -1;
  hipLaunchKernelGGL(ref_copy_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                     (uint64_t)dst, (uint64_t)src, n_bytes / 16);
  return hipGetLastError() == hipSuccess ? 0 : -9;
}

}  // extern "C"
