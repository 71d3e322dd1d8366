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
//   3. a piece is copied by its wave with buffer loads (at whatever
//      alignment the source has: gfx950 runs the HSA unaligned-access mode)
//      and 16-byte destination-aligned buffer stores, both non-temporal;
//      rounds of 4 x `unroll` 1 KiB rows, the next round's loads issued
//      before the current round's stores (see copy_span); the at most 15
//      bytes before the first and after the last aligned destination vector
//      are copied byte by byte, so no store ever touches a byte outside the
//      request;
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

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;
// Global address space (1): plain global_load/global_store instead of flat.
#define GLOBAL __attribute__((address_space(1)))

// Cache policy of the body's buffer accesses (gfx950 bits: 1 = sc0, 2 = nt,
// 16 = sc1).  Neither side is touched again by the copy, so the source is
// read non-temporally and the destination written non-temporally at device
// scope.
constexpr int kLoadPolicy = 2;
constexpr int kStorePolicy = 18;
// Pieces of at most this many vector bytes take body_small.
constexpr uint32_t kSmallPiece = 8192;

// A buffer resource over [base, base + bytes): accesses at or past `bytes`
// read zero and write nothing (the hardware's range check), which lets the
// body run whole rounds without clamping its last one.  base and bytes are
// the same in every lane; base may have any alignment (gfx950 runs the HSA
// unaligned-access mode).
__device__ __forceinline__ rsrc_t span_rsrc(uint64_t base, uint32_t bytes) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
  return __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), (short)0,
                                           (int)__builtin_amdgcn_readfirstlane(bytes),
                                           0x00020000);
}

__device__ __forceinline__ v4i bload(rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kLoadPolicy);
}
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, v4i v) {
  __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, kStorePolicy);
}

// nb bytes (a multiple of 16) from rs to rd in rounds of U vector rows (1 KiB
// per row), two rounds in flight: round k + 1 is loaded before round k is
// stored, so a wave never waits for a round's loads with nothing else
// outstanding.  Offsets past nb read zero and store nothing.
template <int U>
__device__ __forceinline__ void body(rsrc_t rs, rsrc_t rd, uint32_t nb, uint32_t lane) {
  constexpr uint32_t R = 1024u * U;
  const uint32_t l16 = 16u * lane;
  v4i a[U], c[U];
#pragma unroll
  for (int k = 0; k < U; k++) a[k] = bload(rs, l16 + 1024u * k);
  for (uint32_t b = 0; b < nb; b += 2 * R) {
#pragma unroll
    for (int k = 0; k < U; k++) c[k] = bload(rs, b + R + l16 + 1024u * k);
#pragma unroll
    for (int k = 0; k < U; k++) bstore(rd, b + l16 + 1024u * k, a[k]);
#pragma unroll
    for (int k = 0; k < U; k++) a[k] = bload(rs, b + 2 * R + l16 + 1024u * k);
#pragma unroll
    for (int k = 0; k < U; k++) bstore(rd, b + R + l16 + 1024u * k, c[k]);
  }
}

// Small pieces (a halo row, the tail of a request) with plain global
// accesses: rounds of 4 vector rows, indices past the last vector clamped to
// it (a repeated vector rewrites equal bytes), stores non-temporal.  On the
// halo exchange (rows of 5,632 B) the buffer body took 159-168 us per
// exchange against 154 us for this one.
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef v4u v4u_any __attribute__((aligned(1)));  // 16 bytes at any alignment
__device__ __forceinline__ void body_small(uint64_t d, uint64_t s, uint32_t nv, uint32_t lane) {
  for (uint32_t b = 0; b < nv; b += 256) {
    uint64_t o[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint32_t i = b + lane + 64u * k;
      o[k] = 16ull * (i < nv ? i : nv - 1);
    }
    v4u r[4];
#pragma unroll
    for (int k = 0; k < 4; k++) r[k] = *(const GLOBAL v4u_any *)(s + o[k]);
#pragma unroll
    for (int k = 0; k < 4; k++) __builtin_nontemporal_store(r[k], (GLOBAL v4u *)(d + o[k]));
  }
}

// Copy destination bytes [lo, hi) from source address s (the source byte of
// lo) with one wavefront: the 16-byte destination vectors [a0, a1) by body<U>
// (loads at the source's own alignment; body_small for at most 8 KiB of
// vectors), and the at most 15 head bytes
// [lo, a0) and 15 tail bytes [a1, hi) one by one.  Every lane copies one byte
// (lanes 0-15 the head bytes, 16-31 the tail bytes, repeating the last one of
// a range, or byte lo when a range is empty; the other lanes byte lo), so
// repeated stores write equal values inside the piece; the byte is loaded
// before the vectors and stored after them, so its latency overlaps theirs.
// A piece is at most 1 GiB (the chunk limit), so offsets inside it fit 32
// bits.
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
  const uint32_t nb = (uint32_t)(a1 - a0);
  if (nb > kSmallPiece)
    body<U>(span_rsrc(s + nh, nb), span_rsrc(a0, nb), nb, lane);
  else if (nb)
    body_small(a0, s + nh, nb >> 4, lane);
  if (bytes) *(GLOBAL unsigned char *)(lo + bo) = byte;
}

__device__ __forceinline__ void copy_range(uint64_t lo, uint64_t hi, uint64_t s, uint32_t unroll,
                                           uint32_t lane) {
  // rounds of 4 x unroll rows (1 KiB each), two rounds in flight: 32 KiB
  // per wave at unroll 4 (on the batched workload 1.5-2 % faster than
  // 16 KiB; byte-misaligned sources of many MiB run better at unroll 2)
  if (unroll >= 4)
    copy_span<16>(lo, hi, s, lane);
  else
    copy_span<8>(lo, hi, s, lane);
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
