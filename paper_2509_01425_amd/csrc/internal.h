// internal.h -- structures shared by the host runtime and the gfx950 kernels
// of the copy engine.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hicr {

constexpr int kCopyBlock = 256;         // threads per copy workgroup (4 waves)
constexpr int kScanBlock = 1024;        // threads of the one scan workgroup
constexpr uint32_t kMaxLdsDescs = 4096; // requests scanned into LDS by every copy workgroup
constexpr uint32_t kTile = 4096;        // requests per tile of a scanned table
constexpr uint32_t kMaxTiles = 4096;    // tiles per launch over a scanned table
constexpr uint32_t kLineBytes = 128;    // interior piece boundaries are line aligned
constexpr uint32_t kMinSplit = 1024;    // never split a request below 1 KiB pieces

// Device-side batch: structure of arrays, uploaded in one copy.  Addresses
// are already resolved from (slot, offset) on the host.
struct DevBatch {
  const uint64_t *dst;   // [n] destination byte address
  const uint64_t *src;   // [n] source byte address
  const uint64_t *size;  // [n] bytes
  const uint64_t *slots; // [n] dst_slot | (uint64_t)src_slot << 32
  uint32_t n;
};

// Schedule as the kernel sees it.
struct DevSched {
  uint32_t chunk, wgs, unroll, cls;
};

// ceil(a / b), in 32-bit arithmetic when both fit (a 64-bit division is
// several times longer on the GPU).
__host__ __device__ inline uint64_t div_up(uint64_t a, uint64_t b) {
  if (a == 0) return 0;
  if (((a | b) >> 32) == 0) return 1 + ((uint32_t)a - 1) / (uint32_t)b;
  return 1 + (a - 1) / b;
}

// Piece length for one request under (chunk, wgs): pieces start at line
// boundaries of the destination (except the first), so a piece never shares
// a 16-byte store with its neighbour inside one request.
__host__ __device__ inline uint64_t piece_len(uint64_t dst, uint64_t size, uint32_t chunk,
                                              uint32_t wgs) {
  uint64_t span = dst + size - (dst & ~(uint64_t)(kLineBytes - 1));
  uint64_t L = chunk;
  if (wgs > 1 && span < (uint64_t)wgs * chunk) {
    uint64_t per = div_up(span, wgs);
    per = (per + kLineBytes - 1) & ~(uint64_t)(kLineBytes - 1);
    if (per < kMinSplit) per = kMinSplit;
    if (per < L) L = per;
  }
  return L;
}

__host__ __device__ inline uint64_t piece_count(uint64_t dst, uint64_t size, uint32_t chunk,
                                                uint32_t wgs) {
  if (size == 0) return 1;  // a zero-byte request still completes (and counts) once
  uint64_t span = dst + size - (dst & ~(uint64_t)(kLineBytes - 1));
  return div_up(span, piece_len(dst, size, chunk, wgs));
}

// Launch the fused copy kernel over one sub-batch (n <= kMaxLdsDescs), piece
// table scanned in LDS by every workgroup.
hipError_t launch_copy(const DevBatch &b, DevSched s, uint32_t grid, hipStream_t stream);
// Scan the pieces of a batch (1 <= n <= kTile * kMaxTiles, fewer than 2^31
// pieces) into a tiled table: ends[0, n) holds each tile's inclusive prefix
// relative to the tile, tile_tot[0, ceil(n / kTile)) the tile totals.
hipError_t launch_scan(const DevBatch &b, DevSched s, uint32_t *ends, uint32_t *tile_tot,
                       hipStream_t stream);
// Launch the copy kernel over a batch whose table launch_scan has written.
hipError_t launch_copy_mem(const DevBatch &b, DevSched s, const uint32_t *ends,
                           const uint32_t *tile_tot, uint32_t grid, hipStream_t stream);
// Raise the slot counters of n requests (slots[i] = dst | src << 32); queued
// after the copy launches of the same requests on the same stream.  When the
// launch is a single workgroup (n <= 1,024) and done is not null, the kernel
// ends by storing seq to *done (pinned host memory) and *armed is set.
hipError_t launch_count(const uint64_t *slots, uint64_t n, uint64_t *counters, hipStream_t stream,
                        uint64_t *done = nullptr, uint64_t seq = 0, bool *armed = nullptr);
// Workgroups of the copy kernel that one CU holds at once.
int copy_occupancy(int *wgs_per_cu);

}  // namespace hicr
