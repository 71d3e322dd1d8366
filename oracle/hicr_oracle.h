/*
 * hicr_oracle.h -- CPU oracle for the HiCR communication-manager data path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously correct model
 * of what the GPU library computes.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * constant table or helper with the GPU library; the return-code values are
 * an interface that both sides state independently.
 *
 * Passages followed (HiCR paper, arXiv 2509.01425):
 *   Sec. 3.1.2  memory spaces;
 *   Sec. 3.1.3  local memory slots: registration of an existing allocation
 *               by (address, size, memory space);
 *   Sec. 3.1.4  memcpy(dst, dstOff, src, srcOff, size); rejection of an
 *               unsupported memory-space pair; completion only through a
 *               fence that waits for the expected number of incoming and
 *               outgoing transfers;
 *   Sec. 4.3    Channels frontend: circular buffers pre-allocated at the
 *               consumer, a producer that may not push into a full buffer
 *               until the consumer signals consumption; SPSC and MPSC, the
 *               latter locking (one shared buffer, exclusive access) or
 *               non-locking (one buffer per producer).
 */
#ifndef HICR_ORACLE_H
#define HICR_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ERANGE (-2)
#define OR_EBADSLOT (-3)
#define OR_EUNSUPPORTED (-4)
#define OR_EAGAIN (-5)
#define OR_ENOMEM (-6)
#define OR_ETIMEDOUT (-7)
#define OR_EHAZARD (-8)

/* One memcpy request, Sec. 3.1.4 argument order (dst, dstOff, src, srcOff, size). */
typedef struct {
  uint32_t dst_slot;
  uint32_t src_slot;
  uint64_t dst_off;
  uint64_t src_off;
  uint64_t size;
} or_desc;

typedef struct or_ctx or_ctx;

/* pair_mask: bit (2*dst_space + src_space) set <=> that pair is supported. */
or_ctx *or_ctx_create(uint32_t pair_mask);
void or_ctx_destroy(or_ctx *c);

int or_slot_register(or_ctx *c, void *base, uint64_t size, uint32_t space, uint32_t *out);
int or_slot_deregister(or_ctx *c, uint32_t slot);
int or_slot_counters(const or_ctx *c, uint32_t slot, uint64_t *sent, uint64_t *recv);

int or_check_desc(const or_ctx *c, const or_desc *d);
int or_memcpy(or_ctx *c, uint32_t dst, uint64_t dst_off, uint32_t src, uint64_t src_off,
              uint64_t size);
int or_memcpy_batch(or_ctx *c, const or_desc *d, uint64_t n, uint64_t *bad_index);
int or_count_batch(or_ctx *c, const or_desc *d, uint64_t n, uint64_t *bad_index);
int or_hazard_check(const or_ctx *c, const or_desc *d, uint64_t n, uint64_t *bad_a,
                    uint64_t *bad_b);
int or_fence(or_ctx *c);
int or_fence_slot(const or_ctx *c, uint32_t slot, uint64_t exp_sent, uint64_t exp_recv);

/* Byte-loop copy used by every memcpy above (exposed for the libc pin). */
void or_copy_bytes(unsigned char *dst, const unsigned char *src, uint64_t n);

/* ---- fixed-size SPSC channel: C tokens of T bytes ---------------------- */
typedef struct {
  unsigned char *ring; /* C*T bytes, owned by the caller */
  uint64_t C, T;
  uint64_t head, tail; /* monotone token counters */
} or_fchan;

int or_fchan_init(or_fchan *ch, void *ring, uint64_t C, uint64_t T);
int or_fchan_push(or_fchan *ch, const void *src, uint64_t k);
int or_fchan_peek(const or_fchan *ch, uint64_t i, uint64_t *ring_off);
int or_fchan_pop(or_fchan *ch, uint64_t n);
uint64_t or_fchan_depth(const or_fchan *ch);

/* ---- variable-size SPSC channel: P payload bytes, E size entries ------- */
typedef struct {
  unsigned char *payload; /* P bytes, owned by the caller */
  uint64_t P;
  uint64_t *sizes; /* E entries, owned by the caller */
  uint32_t *tags;  /* E producer tags (locking MPSC) or NULL */
  uint64_t E;
  uint64_t hm, tm, hb, tb; /* monotone message and byte counters */
} or_vchan;

int or_vchan_init(or_vchan *ch, void *payload, uint64_t P, uint64_t *sizes, uint32_t *tags,
                  uint64_t E);
int or_vchan_push(or_vchan *ch, uint32_t producer, const void *src, uint64_t s);
int or_vchan_peek(const or_vchan *ch, uint64_t i, uint64_t *ring_off, uint64_t *size,
                  uint32_t *producer);
int or_vchan_read(const or_vchan *ch, uint64_t i, void *dst);
int or_vchan_pop(or_vchan *ch, uint64_t n);
void or_vchan_depth(const or_vchan *ch, uint64_t *msgs, uint64_t *bytes);

/* Test harness (no paper passage of its own): drive ring `ch` with one
 * sequential schedule.  Push number t (t = 0 .. n-1) is made by producer
 * order[t] (< K) and carries that producer's next message: bytes
 * srcs[p] + offs[p][k] .. + sizes[p][k], k counting the producer's pushes
 * (k < counts[p], else OR_EINVAL).
 * A push that finds no room first consumes the oldest message -- read into
 * outs[q] at byte used[q], q the producer its entry names (0 untagged), then
 * popped -- and is retried; at the end the ring is drained the same way.
 * used[0 .. K) must start at zero.  Returns OR_OK or the first error of a
 * push, read or pop (OR_EINVAL for a producer id >= K). */
int or_vchan_replay(or_vchan *ch, uint32_t K, const uint32_t *order, uint64_t n,
                    const unsigned char *const *srcs, const uint64_t *const *offs,
                    const uint64_t *const *sizes, const uint64_t *counts,
                    unsigned char *const *outs, uint64_t *used);

#ifdef __cplusplus
}
#endif
#endif
