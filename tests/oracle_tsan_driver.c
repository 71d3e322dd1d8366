/* oracle_tsan_driver.c -- the oracle under ThreadSanitizer, used the way the
 * benchmark's all-core CPU baseline uses it: every thread creates its own
 * context, registers the same two host buffers (a shared read-only source,
 * a destination of which each thread writes its own ranges), copies its
 * share of the requests and fences; then every thread replays a
 * variable-size ring of its own (one SPSC stream, as the channel baseline
 * does).  Built with gcc -fsanitize=thread by tests/test_oracle_tsan.py; a
 * data race between contexts would be reported and fail the test.
 *
 * argv[1] == "overlap" plants a race in this driver, not in the oracle: two
 * threads copy into the same destination range, so the test can confirm
 * that the build reports races at all.
 * Exit status: 0 when every byte and counter is as expected. */
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hicr_oracle.h"

enum { kThreads = 8, kReqPerThread = 64, kRegion = 1 << 16, kMsgs = 200, kRing = 4096 };

static unsigned char *g_src, *g_dst;
static int g_overlap;

static uint64_t mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

typedef struct {
  int t;
  int ok;
} job;

static void *run(void *arg) {
  job *j = (job *)arg;
  const int t = j->t;
  j->ok = 0;
  /* memcpy requests: thread t writes only destination region t (region 0 for
   * every thread when a race is planted) */
  or_ctx *c = or_ctx_create(0xFu);
  if (!c) return NULL;
  uint32_t sd, ss;
  const uint64_t total = (uint64_t)kThreads * kRegion;
  if (or_slot_register(c, g_dst, total, 0, &sd) != OR_OK ||
      or_slot_register(c, g_src, total, 0, &ss) != OR_OK)
    return NULL;
  or_desc d[kReqPerThread];
  const uint64_t region = g_overlap && t < 2 ? 0 : (uint64_t)t * kRegion;
  const uint64_t slice = kRegion / kReqPerThread;
  for (int k = 0; k < kReqPerThread; k++) {
    const uint64_t h = mix((uint64_t)t * 1000 + (uint64_t)k);
    d[k].dst_slot = sd;
    d[k].src_slot = ss;
    d[k].dst_off = region + (uint64_t)k * slice + h % 8;
    d[k].size = 1 + (h >> 8) % (slice - 8);
    d[k].src_off = (h >> 24) % (total - d[k].size);
  }
  uint64_t bad = 0;
  if (or_memcpy_batch(c, d, kReqPerThread, &bad) != OR_OK || or_fence(c) != OR_OK) return NULL;
  uint64_t sent = 0, recv = 0;
  if (or_slot_counters(c, sd, &sent, &recv) != OR_OK || recv != kReqPerThread) return NULL;
  if (!g_overlap)
    for (int k = 0; k < kReqPerThread; k++)
      if (memcmp(g_dst + d[k].dst_off, g_src + d[k].src_off, d[k].size) != 0) return NULL;
  or_ctx_destroy(c);

  /* one SPSC stream through a variable-size ring of this thread's own */
  unsigned char *payload = malloc(kRing), *in = malloc(kMsgs * 64), *out = malloc(kMsgs * 64);
  uint64_t *ring_sizes = malloc(sizeof(uint64_t) * 16), offs[kMsgs], szs[kMsgs];
  uint32_t *tags = malloc(sizeof(uint32_t) * 16), *order = malloc(sizeof(uint32_t) * kMsgs);
  if (!payload || !in || !out || !ring_sizes || !tags || !order) return NULL;
  uint64_t pos = 0;
  for (int k = 0; k < kMsgs; k++) {
    szs[k] = mix((uint64_t)t * 7777 + (uint64_t)k) % 64;
    offs[k] = pos;
    pos += szs[k];
    order[k] = 0;
  }
  for (uint64_t i = 0; i < pos; i++) in[i] = (unsigned char)mix(i + (uint64_t)t);
  or_vchan ch;
  if (or_vchan_init(&ch, payload, kRing, ring_sizes, tags, 16) != OR_OK) return NULL;
  const unsigned char *srcs[1] = {in};
  const uint64_t *offp[1] = {offs}, *szp[1] = {szs};
  const uint64_t counts[1] = {kMsgs};
  unsigned char *outs[1] = {out};
  uint64_t used[1] = {0};
  if (or_vchan_replay(&ch, 1, order, kMsgs, srcs, offp, szp, counts, outs, used) != OR_OK ||
      used[0] != pos || memcmp(in, out, pos) != 0)
    return NULL;
  free(payload);
  free(in);
  free(out);
  free(ring_sizes);
  free(tags);
  free(order);
  j->ok = 1;
  return NULL;
}

int main(int argc, char **argv) {
  g_overlap = argc > 1 && strcmp(argv[1], "overlap") == 0;
  const uint64_t total = (uint64_t)kThreads * kRegion;
  g_src = malloc(total);
  g_dst = calloc(total, 1);
  if (!g_src || !g_dst) return 2;
  for (uint64_t i = 0; i < total; i++) g_src[i] = (unsigned char)mix(i);
  pthread_t th[kThreads];
  job jobs[kThreads];
  for (int t = 0; t < kThreads; t++) {
    jobs[t].t = t;
    if (pthread_create(&th[t], NULL, run, &jobs[t]) != 0) return 3;
  }
  int ok = 1;
  for (int t = 0; t < kThreads; t++) {
    pthread_join(th[t], NULL);
    ok &= jobs[t].ok;
  }
  printf("threads %d, all checks %s\n", kThreads, ok ? "passed" : "FAILED");
  return ok ? 0 : 1;
}
