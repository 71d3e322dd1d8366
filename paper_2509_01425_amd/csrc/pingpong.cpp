// pingpong.cpp -- host side of the two-endpoint ping-pong (the paper's Test
// Case 1 on one GPU).
#include <algorithm>
#include <vector>

#include "pingpong.h"
#include "runtime.h"

using namespace hicr;

extern "C" {

int hicr_pingpong(hicr_ctx c, hicr_slot src, hicr_slot dst, hicr_slot ring_a, hicr_slot ring_b,
                  hicr_slot buf, const uint64_t *sizes, uint32_t n_sizes, uint32_t reps,
                  uint32_t wgs_per_endpoint, uint64_t *rtt_ticks) {
  return guarded([&]() -> int {
    if (!c || (n_sizes && (!sizes || !rtt_ticks)) || reps == 0 || reps > 100000) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    uint64_t smax = 0;
    for (uint32_t i = 0; i < n_sizes; i++) smax = std::max(smax, sizes[i]);
    const hicr_slot ids[5] = {src, dst, ring_a, ring_b, buf};
    uint64_t base[5];
    for (int i = 0; i < 5; i++) {
      if (ids[i] >= c->slots.size() || !c->slots[ids[i]].live) return fail(c, HICR_EBADSLOT, "slot");
      const Slot &s = c->slots[ids[i]];
      if (s.space != HICR_MEM_HBM) return fail(c, HICR_EUNSUPPORTED, "slot not in HBM");
      if (s.base % 16) return fail(c, HICR_EINVAL, "slots must be 16-byte aligned");
      if (s.size < smax) return fail(c, HICR_ERANGE, "slot smaller than the largest message");
      base[i] = s.base;
    }
    int occ = 0;
    if (pingpong_occupancy(&occ) != 0 || occ < 1) occ = 1;
    const uint64_t cap = (uint64_t)c->n_cu * occ / 2;
    int rc = flush_pending(c);
    if (rc == HICR_OK) rc = wait_all(c);
    if (rc != HICR_OK) return rc;
    const size_t words = 4 + 2 * (size_t)reps + 1;
    uint64_t *d = nullptr;
    std::vector<uint64_t> h(words);
    if (hipMalloc(&d, words * 8) != hipSuccess) return fail(c, HICR_ENOMEM, "ping-pong words");
    for (uint32_t i = 0; i < n_sizes && rc == HICR_OK; i++) {
      uint64_t W = wgs_per_endpoint;
      // one workgroup copies ~10 GB/s; give every 64 KiB of message its own
      if (W == 0) W = std::max<uint64_t>(1, std::min<uint64_t>(256, sizes[i] >> 16));
      W = std::min<uint64_t>(W, cap);
      PingPongArgs a;
      a.src = base[0];
      a.dst = base[1];
      a.ring_a = base[2];
      a.ring_b = base[3];
      a.buf = base[4];
      a.size = sizes[i];
      a.W = (uint32_t)W;
      a.reps = reps;
      a.ctr = d;
      a.t_start = d + 4;
      a.t_end = d + 4 + reps;
      a.err = reinterpret_cast<uint32_t *>(d + 4 + 2 * reps);
      a.timeout_ticks = 1'000'000'000ull;  // 10 s without progress
      hipError_t e = hipMemsetAsync(d, 0, words * 8, c->stream);
      if (e == hipSuccess) e = launch_pingpong(a, c->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, words * 8, hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) {
        rc = hip_fail(c, e, "ping-pong");
        break;
      }
      if (h[4 + 2 * reps]) {
        rc = fail(c, HICR_ETIMEDOUT, "ping-pong of %llu bytes made no progress",
                  (unsigned long long)sizes[i]);
        break;
      }
      for (uint32_t k = 0; k < reps; k++) rtt_ticks[(size_t)i * reps + k] = h[4 + reps + k] - h[4 + k];
    }
    (void)hipFree(d);
    return rc;
  });
}

}  // extern "C"
