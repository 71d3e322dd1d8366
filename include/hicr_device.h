/* hicr_device.h -- channel endpoints inside a caller's own HIP kernels
 * (HiCR Sec. 4.3, Channels frontend), for persistent kernels that produce or
 * consume messages themselves instead of through hicr_channel_pump.
 *
 * This is a HIP header (device functions), not part of the C ABI.  The host
 * obtains a hicr_dev_ring for one ring of a device-endpoint SPSC or
 * non-locking MPSC channel with hicr_channel_device_view (hicr.h) and passes
 * it to its kernel by value.  One ring has one producer and one consumer; the
 * functions below are called by ONE thread of each side, the payload bytes
 * are moved by as many threads as the caller likes:
 *
 *   producer: hicr_dev_push_reserve -> copy into the span(s) -> barrier of
 *             the copying threads -> hicr_dev_push_commit
 *   consumer: hicr_dev_peek(i) -> copy out of the span(s) -> barrier ->
 *             hicr_dev_pop(n)
 *
 * Nothing blocks: a full ring (reserve) or a missing message (peek, pop)
 * returns HICR_EAGAIN, and the caller retries (Sec. 4.3: the producer may
 * not send until the consumer has freed room).  Counters are the ring's
 * monotone message and byte counters; a commit publishes with an agent-scope
 * release, a pop frees room with an agent-scope release, and reserve / peek
 * acquire what the other side released.  A channel handed to user kernels is
 * not pumped by the library afterwards (hicr_channel_pump -> HICR_EINVAL).
 */
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hicr.h"

/* A writable or readable stretch of one message in the ring payload: the
 * message occupies [addr0, addr0 + len0) then, when it wraps around the ring
 * end, [addr1, addr1 + len1). */
typedef struct {
  uint64_t addr0, len0, addr1, len1;
  uint64_t bytes;  /* len0 + len1 */
  uint64_t seq;    /* message counter of this message */
  uint64_t pos;    /* byte counter of its first byte */
} hicr_dev_span;

/* word offsets in the ring's coordination block (128-byte lines):
 * producer line {messages published, bytes published}, consumer line
 * {messages released, bytes released} */
#define HICR_DEV_TM 0
#define HICR_DEV_TB 1
#define HICR_DEV_HM 16
#define HICR_DEV_HB 17

__device__ inline uint64_t hicr_dev_ld_(const hicr_dev_ring *r, int w) {
  return __hip_atomic_load((uint64_t *)r->coord + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void hicr_dev_st_(const hicr_dev_ring *r, int w, uint64_t v) {
  __hip_atomic_store((uint64_t *)r->coord + w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void hicr_dev_span_at_(const hicr_dev_ring *r, uint64_t pos, uint64_t n,
                                         hicr_dev_span *s) {
  const uint64_t p = pos % r->P;
  const uint64_t first = r->P - p < n ? r->P - p : n;
  s->addr0 = r->payload + p;
  s->len0 = first;
  s->addr1 = r->payload;
  s->len1 = n - first;
  s->bytes = n;
  s->pos = pos;
}

/* Producer: room for a message of `bytes` (at most P) at the ring's tail. */
__device__ inline int hicr_dev_push_reserve(const hicr_dev_ring *r, uint64_t bytes,
                                            hicr_dev_span *s) {
  if (bytes > r->P) return HICR_EINVAL;
  const uint64_t tm = hicr_dev_ld_(r, HICR_DEV_TM), tb = hicr_dev_ld_(r, HICR_DEV_TB);
  const uint64_t hm = hicr_dev_ld_(r, HICR_DEV_HM), hb = hicr_dev_ld_(r, HICR_DEV_HB);
  if (tm - hm >= r->E || tb - hb + bytes > r->P) return HICR_EAGAIN;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the consumer's reads of that room are done
  hicr_dev_span_at_(r, tb, bytes, s);
  s->seq = tm;
  return HICR_OK;
}

/* Producer: publish the reserved message once every byte of it is written
 * (the writing threads have passed a barrier with the calling thread). */
__device__ inline void hicr_dev_push_commit(const hicr_dev_ring *r, const hicr_dev_span *s) {
  ((uint64_t *)r->entries)[s->seq % r->E] = s->bytes | ((uint64_t)r->producer << 48);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  hicr_dev_st_(r, HICR_DEV_TB, s->pos + s->bytes);
  hicr_dev_st_(r, HICR_DEV_TM, s->seq + 1);
}

/* Consumer: where the i-th oldest unreleased message lies. */
__device__ inline int hicr_dev_peek(const hicr_dev_ring *r, uint64_t i, hicr_dev_span *s) {
  const uint64_t tm = hicr_dev_ld_(r, HICR_DEV_TM);
  const uint64_t hm = hicr_dev_ld_(r, HICR_DEV_HM), hb = hicr_dev_ld_(r, HICR_DEV_HB);
  if (i >= tm - hm) return HICR_EAGAIN;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // entries and payload published up to tm
  const uint64_t *ent = (const uint64_t *)r->entries;
  uint64_t pos = hb;
  for (uint64_t k = 0; k < i; k++) pos += ent[(hm + k) % r->E] & ((1ull << 48) - 1);
  hicr_dev_span_at_(r, pos, ent[(hm + i) % r->E] & ((1ull << 48) - 1), s);
  s->seq = hm + i;
  return HICR_OK;
}

/* Consumer: free the n oldest messages once every read of them is done (the
 * reading threads have passed a barrier with the calling thread). */
__device__ inline int hicr_dev_pop(const hicr_dev_ring *r, uint64_t n) {
  const uint64_t tm = hicr_dev_ld_(r, HICR_DEV_TM);
  const uint64_t hm = hicr_dev_ld_(r, HICR_DEV_HM), hb = hicr_dev_ld_(r, HICR_DEV_HB);
  if (n > tm - hm) return HICR_EAGAIN;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const uint64_t *ent = (const uint64_t *)r->entries;
  uint64_t b = hb;
  for (uint64_t k = 0; k < n; k++) b += ent[(hm + k) % r->E] & ((1ull << 48) - 1);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  hicr_dev_st_(r, HICR_DEV_HB, b);
  hicr_dev_st_(r, HICR_DEV_HM, hm + n);
  return HICR_OK;
}
