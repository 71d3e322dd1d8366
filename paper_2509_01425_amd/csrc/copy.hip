// copy.hip -- fused batched memcpy for gfx950 (CDNA4).
//
// One launch moves a batch of memcpy(dst, dstOff, src, srcOff, size)
// requests (HiCR Sec. 3.1.4) with a persistent grid:
//   1. the batch becomes one global index space of pieces: an inclusive
//      prefix scan of the pieces per request.  A batch of at most 4,096
//      requests is scanned by every workgroup into LDS (wavefront scans with
//      __shfl_up, then a cross-wave carry); a larger one is scanned once, by
//      scan_kernel, one workgroup per tile of 4,096 requests (the tile's
//      prefix staged in LDS, written to device memory with the tile total),
//      and every copy workgroup scans only the tile totals into LDS;
//   2. every wavefront is an independent worker.  Against an LDS table,
//      wave w of workgroup g takes pieces 4g + w, 4g + w + 4G, ... and finds
//      each piece's request by a 64-ary ballot search (two ballots for 4,096
//      requests).  Against the tiled table, every wavefront takes one
//      contiguous range of pieces, searches once for its first request (tile,
//      then request inside the tile) and walks forward request by request;
//   3. a piece is copied by its wave with 16-byte destination-aligned vector
//      stores and 16-byte loads at whatever alignment the source has (the HSA
//      ABI runs gfx950 in unaligned-access mode), `unroll` vectors in flight
//      per lane, branch-free (see copy_span); the at most 15 bytes before
//      the first and after the last aligned destination vector are copied
//      byte by byte, so no store ever touches a byte outside the request;
//   4. completion counting is a separate small kernel (count.hip) queued
//      behind the copy launches of a submission on the same stream: the
//      kernel boundary makes every copied byte visible before any counter
//      rises, so the copy kernel needs no per-workgroup release (an
//      agent-scope release writes back the whole L2 of the XCD, and one per
//      workgroup cost more than the copy itself on batches of small
//      requests).  count_kernel sums the counts per slot in LDS first, so a
//      slot named by many requests costs one device atomic per counter.
#include "internal.h"

namespace hicr {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef v4u v4u_any __attribute__((aligned(1)));  // 16 bytes at any alignment
// Global address space (1): plain global_load/global_store instead of flat.
#define GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ v4u load16(uint64_t a) { return *(const GLOBAL v4u_any *)a; }

// Body stores are non-temporal: the destination is not read again by this
// kernel, and streaming it past the caches measured ~2% faster on gfx950.
__device__ __forceinline__ void store16(uint64_t a, v4u v) {
  __builtin_nontemporal_store(v, (GLOBAL v4u *)a);
}

// First index i in [0, n) with ends[i] > q (ends strictly increasing, q <
// ends[n-1]; ends in LDS or device memory).  Every lane of the wave returns
// the same value.
template <typename Ends>
__device__ __forceinline__ uint32_t find_piece_owner(Ends ends, uint32_t n, uint32_t q,
                                                     uint32_t lane) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 64) {
    uint32_t step = (hi - lo + 63) >> 6;
    uint32_t idx = lo + (lane + 1) * step - 1;
    bool gt = (idx >= hi - 1) ? true : (ends[idx] > q);
    uint64_t m = __ballot(gt);
    uint32_t f = (uint32_t)__ffsll((unsigned long long)m) - 1;
    uint32_t nlo = lo + f * step;
    uint32_t nhi = lo + (f + 1) * step;
    hi = nhi < hi ? nhi : hi;
    lo = nlo;
  }
  uint32_t idx = lo + lane;
  bool gt = (idx >= hi - 1) ? true : (ends[idx] > q);
  uint64_t m = __ballot(gt);
  return lo + (uint32_t)__ffsll((unsigned long long)m) - 1;
}

// Copy destination bytes [lo, hi) from source address s (the source byte of
// lo) with one wavefront: 16-byte destination-aligned vectors, `unroll`
// (U) per lane in flight, and the at most 15 head bytes [lo, a0) and 15 tail
// bytes [a1, hi) one by one.  The code has no per-lane branch: past the last
// vector a lane copies the last vector again, and every lane copies one byte
// (lanes 0-15 the head bytes, 16-31 the tail bytes, repeating the last one
// of a range, or byte lo when a range is empty; the other lanes byte lo), so
// repeated stores write equal values inside the piece.  A bounds test per
// access made the compiler wait for each access of a partial round in turn
// (four memory latencies for the last round of a piece instead of one); the
// byte is loaded before the vectors and stored after them, so its latency
// overlaps theirs.
template <int U>
__device__ __forceinline__ void copy_span(uint64_t lo, uint64_t hi, uint64_t s, uint32_t lane) {
  uint64_t a0 = (lo + 15) & ~(uint64_t)15;
  if (a0 > hi) a0 = hi;
  uint64_t a1 = hi & ~(uint64_t)15;
  if (a1 < a0) a1 = a0;
  const uint64_t nh = a0 - lo, nt = hi - a1;
  uint64_t bo = 0;  // this lane's byte, as an offset from lo
  if (lane < 16)
    bo = nh ? (lane < nh ? lane : nh - 1) : 0;
  else if (lane < 32)
    bo = nt ? (a1 - lo) + (lane - 16 < nt ? lane - 16 : nt - 1) : 0;
  // (lo and hi are the same in every lane: a piece without head or tail
  // bytes, such as an aligned row, skips the byte copy altogether)
  const bool bytes = (nh | nt) != 0;
  unsigned char byte = 0;
  if (bytes) byte = *(const GLOBAL unsigned char *)(s + bo);
  const uint64_t nv = (a1 - a0) >> 4;
  const uint64_t s16 = s + nh;
  constexpr uint64_t step = 64ull * U;
  for (uint64_t base = 0; base < nv; base += step) {
    uint64_t o[U];
#pragma unroll
    for (int k = 0; k < U; k++) {
      const uint64_t i = base + lane + 64ull * k;
      o[k] = 16 * (i < nv ? i : nv - 1);
    }
    v4u r[U];
#pragma unroll
    for (int k = 0; k < U; k++) r[k] = load16(s16 + o[k]);
#pragma unroll
    for (int k = 0; k < U; k++) store16(a0 + o[k], r[k]);
  }
  if (bytes) *(GLOBAL unsigned char *)(lo + bo) = byte;
}

__device__ __forceinline__ void copy_range(uint64_t lo, uint64_t hi, uint64_t s, uint32_t unroll,
                                           uint32_t lane) {
  if (unroll >= 4)
    copy_span<4>(lo, hi, s, lane);
  else
    copy_span<2>(lo, hi, s, lane);
}

// Piece j (of length L) of the request dst <- src, size bytes: pieces start
// at line boundaries of the destination, the first and last clipped to the
// request.
__device__ __forceinline__ void copy_piece(uint64_t dst, uint64_t src, uint64_t size, uint64_t L,
                                           uint32_t j, uint32_t unroll, uint32_t lane) {
  const uint64_t base = dst & ~(uint64_t)(kLineBytes - 1);
  uint64_t lo = base + (uint64_t)j * L, hi = lo + L;
  if (lo < dst) lo = dst;
  if (hi > dst + size) hi = dst + size;
  if (lo < hi) copy_range(lo, hi, src + (lo - dst), unroll, lane);
}

// Inclusive prefix scan, in place, of v[0, m) in LDS by a whole workgroup
// of B threads: every thread sums a run of consecutive entries, the run sums
// are scanned per wavefront with __shfl_up, wsum[] carries across
// wavefronts, and every thread rewrites its run.  Ends with a barrier.
template <int B>
__device__ __forceinline__ void block_scan(uint32_t *v, uint32_t m, uint32_t *wsum) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t per = (m + B - 1) / B;
  const uint32_t k0 = min(tid * per, m), k1 = min(k0 + per, m);
  uint32_t sum = 0;
  for (uint32_t k = k0; k < k1; k++) sum += v[k];
  uint32_t inc = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(inc, o, 64);
    if (lane >= (uint32_t)o) inc += t;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t run = inc - sum;
  for (uint32_t w = 0; w < wave; w++) run += wsum[w];
  for (uint32_t k = k0; k < k1; k++) {
    run += v[k];
    v[k] = run;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kCopyBlock) void copy_kernel(DevBatch b, DevSched s) {
  __shared__ uint32_t ends[kMaxLdsDescs];
  __shared__ uint32_t wsum[kCopyBlock / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t n = b.n;

  // 1. pieces per request, then an inclusive block scan in LDS
  for (uint32_t i = tid; i < n; i += kCopyBlock)
    ends[i] = (uint32_t)piece_count(b.dst[i], b.size[i], s.chunk, s.wgs);
  __syncthreads();
  block_scan<kCopyBlock>(ends, n, wsum);
  const uint32_t total = n ? ends[n - 1] : 0;

  // 2-3. persistent loop over pieces, one wavefront per piece
  constexpr uint32_t kWaves = kCopyBlock / 64;
  const uint32_t first = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + wave);
  const uint32_t stride = gridDim.x * kWaves;
  for (uint32_t q = first; q < total; q += stride) {
    uint32_t i = __builtin_amdgcn_readfirstlane(find_piece_owner(ends, n, q, lane));
    uint32_t j = q - (i ? ends[i - 1] : 0u);
    const uint64_t dst = b.dst[i], src = b.src[i], size = b.size[i];
    copy_piece(dst, src, size, piece_len(dst, size, s.chunk, s.wgs), j, s.unroll, lane);
  }
}

// Table of a large batch, one workgroup per tile of kTile requests: the
// tile's piece counts are loaded (all of a thread's loads in flight at
// once), counted into LDS, scanned there, and written out as the tile's
// inclusive prefix (relative to the tile's first piece) with the tile's
// total in tile_tot[tile].
__global__ __launch_bounds__(kScanBlock) void scan_kernel(DevBatch b, DevSched s, uint32_t *ends,
                                                          uint32_t *tile_tot) {
  constexpr int kPer = kTile / kScanBlock;
  __shared__ uint32_t cnt[kTile];
  __shared__ uint32_t wsum[kScanBlock / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t i0 = blockIdx.x * kTile, m = min(b.n - i0, kTile);
  uint64_t dv[kPer], zv[kPer];
#pragma unroll
  for (int r = 0; r < kPer; r++) {
    const uint32_t k = tid + r * kScanBlock;
    dv[r] = k < m ? b.dst[i0 + k] : 0;
    zv[r] = k < m ? b.size[i0 + k] : 0;
  }
#pragma unroll
  for (int r = 0; r < kPer; r++) {
    const uint32_t k = tid + r * kScanBlock;
    if (k < m) cnt[k] = (uint32_t)piece_count(dv[r], zv[r], s.chunk, s.wgs);
  }
  __syncthreads();
  block_scan<kScanBlock>(cnt, m, wsum);
  for (uint32_t k = tid; k < m; k += kScanBlock) ends[i0 + k] = cnt[k];
  if (tid == 0) tile_tot[blockIdx.x] = cnt[m - 1];
}

// Copy against the tiled table in device memory.  Every workgroup first
// scans the tile totals into LDS (at most kMaxTiles of them), so piece q's
// global index is tile_base(tile) + local prefix.  Wavefront w of the W in
// the grid takes pieces [total * w / W, total * (w + 1) / W), finds the
// request of its first piece (64-ary search over the tile bases, then over
// that tile's prefix) and walks forward from there: every request has at
// least one piece, so the walk advances one request at a time, and the next
// request's descriptor is loaded before the current piece is copied.
__global__ __launch_bounds__(kCopyBlock) void copy_kernel_mem(DevBatch b, DevSched s,
                                                              const uint32_t *ends_in,
                                                              const uint32_t *tile_tot) {
  __shared__ uint32_t tiles[kMaxTiles];
  __shared__ uint32_t wsum[kCopyBlock / 64];
  const GLOBAL uint32_t *ends = (const GLOBAL uint32_t *)ends_in;
  constexpr uint32_t kWaves = kCopyBlock / 64;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t n = b.n, nt = (n + kTile - 1) / kTile;
  for (uint32_t k = threadIdx.x; k < nt; k += kCopyBlock) tiles[k] = tile_tot[k];
  __syncthreads();
  block_scan<kCopyBlock>(tiles, nt, wsum);
  const uint64_t total = tiles[nt - 1];
  const uint64_t W = (uint64_t)gridDim.x * kWaves;
  const uint64_t gw = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6));
  uint32_t q = (uint32_t)(total * gw / W);
  const uint32_t q1 = (uint32_t)(total * (gw + 1) / W);
  if (q >= q1) return;
  const uint32_t t = __builtin_amdgcn_readfirstlane(find_piece_owner(tiles, nt, q, lane));
  const uint32_t tb = t ? tiles[t - 1] : 0u, t0 = t * kTile;
  uint32_t i = t0 + __builtin_amdgcn_readfirstlane(
                        find_piece_owner(ends + t0, min(n - t0, kTile), q - tb, lane));
  uint32_t start = tb + (i > t0 ? ends[i - 1] : 0u), end = tb + ends[i];
  uint64_t dst = b.dst[i], src = b.src[i], size = b.size[i];
  for (; q < q1; q++) {
    // piece q + 1 in this range belongs to request i + 1 (< n, since
    // q + 1 < total; checked anyway, so that no table content can send a
    // wavefront past the batch): load its descriptor before copying piece q
    const bool next = q + 1 < q1 && q + 1 >= end && i + 1 < n;
    uint32_t nend = 0;
    uint64_t ndst = 0, nsrc = 0, nsize = 0;
    if (next) {
      const uint32_t nt1 = (i + 1) / kTile;
      nend = (nt1 ? tiles[nt1 - 1] : 0u) + ends[i + 1];
      ndst = b.dst[i + 1];
      nsrc = b.src[i + 1];
      nsize = b.size[i + 1];
    }
    copy_piece(dst, src, size, piece_len(dst, size, s.chunk, s.wgs), q - start, s.unroll, lane);
    if (next) {
      i++;
      start = end;
      end = nend;
      dst = ndst;
      src = nsrc;
      size = nsize;
    }
  }
}

hipError_t launch_copy(const DevBatch &b, DevSched s, uint32_t grid, hipStream_t stream) {
  if (b.n > kMaxLdsDescs || grid == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(kCopyBlock), 0, stream, b, s);
  return hipGetLastError();
}

hipError_t launch_scan(const DevBatch &b, DevSched s, uint32_t *ends, uint32_t *tile_tot,
                       hipStream_t stream) {
  if (b.n == 0 || !ends || !tile_tot || (b.n + kTile - 1) / kTile > kMaxTiles)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(scan_kernel, dim3((b.n + kTile - 1) / kTile), dim3(kScanBlock), 0, stream, b,
                     s, ends, tile_tot);
  return hipGetLastError();
}

hipError_t launch_copy_mem(const DevBatch &b, DevSched s, const uint32_t *ends,
                           const uint32_t *tile_tot, uint32_t grid, hipStream_t stream) {
  if (b.n == 0 || !ends || !tile_tot || grid == 0 || (b.n + kTile - 1) / kTile > kMaxTiles)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_kernel_mem, dim3(grid), dim3(kCopyBlock), 0, stream, b, s, ends,
                     tile_tot);
  return hipGetLastError();
}

int copy_occupancy(int *wgs_per_cu) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, copy_kernel, kCopyBlock,
                                                            0);
}

}  // namespace hicr
