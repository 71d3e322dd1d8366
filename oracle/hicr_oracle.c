/*
 * hicr_oracle.c -- CPU oracle for the HiCR communication-manager data path.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).
 * Plain C, byte loops, no blocking and no reordering beyond what the
 * definitions state.  Every function names the passage it follows.
 */
#include "hicr_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ slots */

typedef struct {
  unsigned char *base;
  uint64_t size;
  uint32_t space;
  int live;
  uint64_t sent; /* outgoing transfers completed (Sec. 3.1.4 fence) */
  uint64_t recv; /* incoming transfers completed */
} or_slot;

struct or_ctx {
  uint32_t pair_mask;
  or_slot *slots;
  uint32_t n, cap;
};

or_ctx *or_ctx_create(uint32_t pair_mask) {
  or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
  if (c) c->pair_mask = pair_mask;
  return c;
}

void or_ctx_destroy(or_ctx *c) {
  if (!c) return;
  free(c->slots);
  free(c);
}

/* Sec. 3.1.3: register an existing allocation by address, size and memory
 * space.  A memory space has non-zero size (Sec. 3.1.2); a slot of size 0 is
 * rejected the same way. */
int or_slot_register(or_ctx *c, void *base, uint64_t size, uint32_t space, uint32_t *out) {
  if (!c || !out || !base || size == 0 || space > 1) return OR_EINVAL;
  if (c->n == c->cap) {
    uint32_t ncap = c->cap ? 2 * c->cap : 16;
    or_slot *s = (or_slot *)realloc(c->slots, (size_t)ncap * sizeof(or_slot));
    if (!s) return OR_ENOMEM;
    c->slots = s;
    c->cap = ncap;
  }
  or_slot *s = &c->slots[c->n];
  s->base = (unsigned char *)base;
  s->size = size;
  s->space = space;
  s->live = 1;
  s->sent = 0;
  s->recv = 0;
  *out = c->n++;
  return OR_OK;
}

int or_slot_deregister(or_ctx *c, uint32_t slot) {
  if (!c || slot >= c->n || !c->slots[slot].live) return OR_EBADSLOT;
  c->slots[slot].live = 0;
  return OR_OK;
}

int or_slot_counters(const or_ctx *c, uint32_t slot, uint64_t *sent, uint64_t *recv) {
  if (!c || slot >= c->n || !c->slots[slot].live) return OR_EBADSLOT;
  if (sent) *sent = c->slots[slot].sent;
  if (recv) *recv = c->slots[slot].recv;
  return OR_OK;
}

/* ----------------------------------------------------------------- memcpy */

void or_copy_bytes(unsigned char *dst, const unsigned char *src, uint64_t n) {
  for (uint64_t j = 0; j < n; j++) dst[j] = src[j];
}

/* Sec. 3.1.4 preconditions of memcpy(dst, dstOff, src, srcOff, size):
 * both slots exist; each (offset, size) lies inside its slot (written so
 * that no sum can overflow); the memory-space pair is supported, otherwise
 * the request is rejected. */
int or_check_desc(const or_ctx *c, const or_desc *d) {
  if (d->dst_slot >= c->n || !c->slots[d->dst_slot].live) return OR_EBADSLOT;
  if (d->src_slot >= c->n || !c->slots[d->src_slot].live) return OR_EBADSLOT;
  const or_slot *ds = &c->slots[d->dst_slot];
  const or_slot *ss = &c->slots[d->src_slot];
  if (d->dst_off > ds->size || d->size > ds->size - d->dst_off) return OR_ERANGE;
  if (d->src_off > ss->size || d->size > ss->size - d->src_off) return OR_ERANGE;
  uint32_t bit = 2u * ds->space + ss->space;
  if (!((c->pair_mask >> bit) & 1u)) return OR_EUNSUPPORTED;
  return OR_OK;
}

/* Effect of one transfer: the bytes move, the source slot counts one
 * outgoing transfer and the destination slot one incoming transfer.  A
 * zero-byte request moves nothing and still counts once. */
static void apply_desc(or_ctx *c, const or_desc *d, int move_bytes) {
  or_slot *ds = &c->slots[d->dst_slot];
  or_slot *ss = &c->slots[d->src_slot];
  if (move_bytes) or_copy_bytes(ds->base + d->dst_off, ss->base + d->src_off, d->size);
  ss->sent += 1;
  ds->recv += 1;
}

int or_memcpy(or_ctx *c, uint32_t dst, uint64_t dst_off, uint32_t src, uint64_t src_off,
              uint64_t size) {
  or_desc d;
  d.dst_slot = dst;
  d.src_slot = src;
  d.dst_off = dst_off;
  d.src_off = src_off;
  d.size = size;
  int rc = or_check_desc(c, &d);
  if (rc != OR_OK) return rc;
  apply_desc(c, &d, 1);
  return OR_OK;
}

/* A batch is n memcpy requests issued back to back in one epoch.  The whole
 * batch is checked first; if any request is invalid nothing is applied and
 * the index of the first bad request is reported.  Otherwise the requests
 * are applied one after another in index order. */
static int batch_common(or_ctx *c, const or_desc *d, uint64_t n, uint64_t *bad, int move) {
  for (uint64_t i = 0; i < n; i++) {
    int rc = or_check_desc(c, &d[i]);
    if (rc != OR_OK) {
      if (bad) *bad = i;
      return rc;
    }
  }
  for (uint64_t i = 0; i < n; i++) apply_desc(c, &d[i], move);
  return OR_OK;
}

int or_memcpy_batch(or_ctx *c, const or_desc *d, uint64_t n, uint64_t *bad) {
  return batch_common(c, d, n, bad, 1);
}

/* The counter effect of a batch alone, for batches whose bytes are too large
 * to hold on the host. */
int or_count_batch(or_ctx *c, const or_desc *d, uint64_t n, uint64_t *bad) {
  return batch_common(c, d, n, bad, 0);
}

/* Completion of a transfer is unobservable before the fence, so within one
 * epoch two requests that write the same byte, or one that writes a byte
 * another reads, race; the result is defined only without such a pair.
 * Plain pairwise check on absolute addresses (slots may alias). */
static int ranges_meet(const unsigned char *a, uint64_t na, const unsigned char *b, uint64_t nb) {
  if (na == 0 || nb == 0) return 0;
  return a < b + nb && b < a + na;
}

int or_hazard_check(const or_ctx *c, const or_desc *d, uint64_t n, uint64_t *bad_a,
                    uint64_t *bad_b) {
  for (uint64_t i = 0; i < n; i++) {
    int rc = or_check_desc(c, &d[i]);
    if (rc != OR_OK) {
      if (bad_a) *bad_a = i;
      if (bad_b) *bad_b = i;
      return rc;
    }
  }
  for (uint64_t i = 0; i < n; i++) {
    const unsigned char *wi = c->slots[d[i].dst_slot].base + d[i].dst_off;
    const unsigned char *ri = c->slots[d[i].src_slot].base + d[i].src_off;
    for (uint64_t j = 0; j < n; j++) {
      const unsigned char *wj = c->slots[d[j].dst_slot].base + d[j].dst_off;
      /* write/write between two different requests */
      int ww = (j > i) && ranges_meet(wi, d[i].size, wj, d[j].size);
      /* request i reads what request j writes (j may equal i) */
      int rw = ranges_meet(ri, d[i].size, wj, d[j].size);
      if (ww || rw) {
        if (bad_a) *bad_a = i;
        if (bad_b) *bad_b = j;
        return OR_EHAZARD;
      }
    }
  }
  return OR_OK;
}

/* The oracle completes every transfer inside the call, so a fence has
 * nothing left to wait for. */
int or_fence(or_ctx *c) { return c ? OR_OK : OR_EINVAL; }

/* Fence on expected counts: satisfied once the slot has seen at least the
 * expected numbers of outgoing and incoming transfers.  With nothing pending
 * an unmet expectation can never be met, which is reported as a time-out. */
int or_fence_slot(const or_ctx *c, uint32_t slot, uint64_t exp_sent, uint64_t exp_recv) {
  uint64_t s, r;
  int rc = or_slot_counters(c, slot, &s, &r);
  if (rc != OR_OK) return rc;
  return (s >= exp_sent && r >= exp_recv) ? OR_OK : OR_ETIMEDOUT;
}

/* --------------------------------------------------- fixed-size SPSC ring */

/* Sec. 4.3: a circular buffer of C tokens at the consumer.  head and tail
 * are monotone token counters; tail - head tokens are in the buffer, and
 * 0 <= tail - head <= C always. */
int or_fchan_init(or_fchan *ch, void *ring, uint64_t C, uint64_t T) {
  if (!ch || !ring || C == 0 || T == 0) return OR_EINVAL;
  ch->ring = (unsigned char *)ring;
  ch->C = C;
  ch->T = T;
  ch->head = 0;
  ch->tail = 0;
  return OR_OK;
}

uint64_t or_fchan_depth(const or_fchan *ch) { return ch->tail - ch->head; }

/* Push k tokens (k*T contiguous source bytes), all or nothing: the producer
 * may not push while the buffer lacks room. */
int or_fchan_push(or_fchan *ch, const void *src, uint64_t k) {
  if (k > ch->C) return OR_EINVAL;
  if (ch->C - (ch->tail - ch->head) < k) return OR_EAGAIN;
  const unsigned char *s = (const unsigned char *)src;
  for (uint64_t t = 0; t < k; t++) {
    uint64_t pos = (ch->tail + t) % ch->C;
    or_copy_bytes(ch->ring + pos * ch->T, s + t * ch->T, ch->T);
  }
  ch->tail += k;
  return OR_OK;
}

/* Ring byte offset of the i-th oldest unconsumed token. */
int or_fchan_peek(const or_fchan *ch, uint64_t i, uint64_t *ring_off) {
  if (i >= ch->tail - ch->head) return OR_EAGAIN;
  *ring_off = ((ch->head + i) % ch->C) * ch->T;
  return OR_OK;
}

/* Consume n tokens: the consumer's notification that frees their room. */
int or_fchan_pop(or_fchan *ch, uint64_t n) {
  if (n > ch->tail - ch->head) return OR_EAGAIN;
  ch->head += n;
  return OR_OK;
}

/* ------------------------------------------------ variable-size SPSC ring */

/* A payload ring of P bytes plus a ring of E message sizes.  Counters:
 * hm/tm messages consumed/produced, hb/tb bytes consumed/produced.  A
 * message is stored at byte positions (tb + j) mod P, so it splits across
 * the end of the ring when it does not fit before it. */
int or_vchan_init(or_vchan *ch, void *payload, uint64_t P, uint64_t *sizes, uint32_t *tags,
                  uint64_t E) {
  if (!ch || !payload || !sizes || P == 0 || E == 0) return OR_EINVAL;
  ch->payload = (unsigned char *)payload;
  ch->P = P;
  ch->sizes = sizes;
  ch->tags = tags;
  ch->E = E;
  ch->hm = ch->tm = ch->hb = ch->tb = 0;
  return OR_OK;
}

void or_vchan_depth(const or_vchan *ch, uint64_t *msgs, uint64_t *bytes) {
  if (msgs) *msgs = ch->tm - ch->hm;
  if (bytes) *bytes = ch->tb - ch->hb;
}

int or_vchan_push(or_vchan *ch, uint32_t producer, const void *src, uint64_t s) {
  if (s > ch->P) return OR_EINVAL;
  if (ch->tm - ch->hm == ch->E) return OR_EAGAIN;
  if ((ch->tb - ch->hb) + s > ch->P) return OR_EAGAIN;
  const unsigned char *b = (const unsigned char *)src;
  for (uint64_t j = 0; j < s; j++) ch->payload[(ch->tb + j) % ch->P] = b[j];
  ch->sizes[ch->tm % ch->E] = s;
  if (ch->tags) ch->tags[ch->tm % ch->E] = producer;
  ch->tb += s;
  ch->tm += 1;
  return OR_OK;
}

int or_vchan_peek(const or_vchan *ch, uint64_t i, uint64_t *ring_off, uint64_t *size,
                  uint32_t *producer) {
  if (i >= ch->tm - ch->hm) return OR_EAGAIN;
  uint64_t start = ch->hb;
  for (uint64_t k = 0; k < i; k++) start += ch->sizes[(ch->hm + k) % ch->E];
  if (ring_off) *ring_off = start % ch->P;
  if (size) *size = ch->sizes[(ch->hm + i) % ch->E];
  if (producer) *producer = ch->tags ? ch->tags[(ch->hm + i) % ch->E] : 0u;
  return OR_OK;
}

/* Copy out the bytes of the i-th oldest message (following the wrap). */
int or_vchan_read(const or_vchan *ch, uint64_t i, void *dst) {
  uint64_t off, s;
  int rc = or_vchan_peek(ch, i, &off, &s, NULL);
  if (rc != OR_OK) return rc;
  unsigned char *o = (unsigned char *)dst;
  for (uint64_t j = 0; j < s; j++) o[j] = ch->payload[(off + j) % ch->P];
  return OR_OK;
}

int or_vchan_pop(or_vchan *ch, uint64_t n) {
  if (n > ch->tm - ch->hm) return OR_EAGAIN;
  for (uint64_t k = 0; k < n; k++) ch->hb += ch->sizes[(ch->hm + k) % ch->E];
  ch->hm += n;
  return OR_OK;
}

/* Consume the oldest message into its producer's output. */
static int consume_oldest(or_vchan *ch, uint32_t K, unsigned char *const *outs, uint64_t *used) {
  uint64_t off, size;
  uint32_t q;
  int rc = or_vchan_peek(ch, 0, &off, &size, &q);
  if (rc != OR_OK) return rc;
  if (q >= K) return OR_EINVAL;
  rc = or_vchan_read(ch, 0, outs[q] + used[q]);
  if (rc != OR_OK) return rc;
  used[q] += size;
  return or_vchan_pop(ch, 1);
}

int or_vchan_replay(or_vchan *ch, uint32_t K, const uint32_t *order, uint64_t n,
                    const unsigned char *const *srcs, const uint64_t *const *offs,
                    const uint64_t *const *sizes, const uint64_t *counts,
                    unsigned char *const *outs, uint64_t *used) {
  uint64_t *next = (uint64_t *)calloc(K ? K : 1, sizeof(uint64_t));
  if (!next) return OR_ENOMEM;
  int rc = OR_OK;
  for (uint64_t t = 0; t < n && rc == OR_OK; t++) {
    const uint32_t p = order[t];
    if (p >= K || next[p] >= counts[p]) {
      rc = OR_EINVAL;
      break;
    }
    const uint64_t k = next[p]++;
    for (;;) {
      rc = or_vchan_push(ch, p, srcs[p] + offs[p][k], sizes[p][k]);
      if (rc != OR_EAGAIN) break;
      rc = consume_oldest(ch, K, outs, used); /* EAGAIN here: empty yet full */
      if (rc != OR_OK) break;
    }
  }
  while (rc == OR_OK && ch->tm != ch->hm) rc = consume_oldest(ch, K, outs, used);
  free(next);
  return rc;
}
