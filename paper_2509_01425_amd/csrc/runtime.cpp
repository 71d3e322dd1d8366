// runtime.cpp -- host side of the communication-manager data path: context,
// slot table, request validation, fused-batch submission and fences.
//
// Slots (HiCR Sec. 3.1.3) live in a host table; requests are validated on
// the host and resolved to absolute device addresses, packed as a structure
// of arrays into pinned staging, uploaded with one asynchronous copy and
// moved by one fused copy launch per (at most 4,096-request) sub-batch.
// Per-slot counters live in device memory and are raised by the copy kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hicr.h"
#include "chan.h"
#include "internal.h"
#include "noalloc.h"
#include "runtime.h"

using namespace hicr;

namespace {

constexpr uint32_t kChunks[3] = {4u << 10, 64u << 10, 1u << 20};
constexpr uint32_t kWgs[2] = {1, 4};
constexpr uint32_t kUnroll[2] = {2, 4};

}  // namespace

namespace hicr {

int fail(hicr_ctx c, int code, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

int hip_fail(hicr_ctx c, hipError_t e, const char *what) {
  return fail(c, HICR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int check_sched(hicr_ctx c, const hicr_sched &s) {
  if (s.chunk_bytes < kLineBytes || s.chunk_bytes > (1u << 30) || s.chunk_bytes % kLineBytes)
    return fail(c, HICR_EINVAL, "chunk_bytes %u: must be a multiple of 128 in [128, 1 GiB]",
                s.chunk_bytes);
  if (s.wgs_per_desc < 1 || s.wgs_per_desc > 64)
    return fail(c, HICR_EINVAL, "wgs_per_desc %u outside [1, 64]", s.wgs_per_desc);
  if (s.unroll != 2 && s.unroll != 4) return fail(c, HICR_EINVAL, "unroll %u not 2 or 4", s.unroll);
  return HICR_OK;
}

int check_desc(hicr_ctx c, const hicr_desc &d) {
  if (d.dst_slot >= c->slots.size() || !c->slots[d.dst_slot].live) return HICR_EBADSLOT;
  if (d.src_slot >= c->slots.size() || !c->slots[d.src_slot].live) return HICR_EBADSLOT;
  const Slot &ds = c->slots[d.dst_slot], &ss = c->slots[d.src_slot];
  if (d.dst_off > ds.size || d.size > ds.size - d.dst_off) return HICR_ERANGE;
  if (d.src_off > ss.size || d.size > ss.size - d.src_off) return HICR_ERANGE;
  if (!(c->pair_mask & HICR_PAIR(ds.space, ss.space))) return HICR_EUNSUPPORTED;
  return HICR_OK;
}

static uint64_t *sub_done_word(hicr_ctx c, const Sub &s) {
  return c->h_done + 8 * (uint64_t)(&s - c->subs);
}

bool any_inflight(hicr_ctx c) {
  if (c->na_inflight) {
    if (hipEventQuery(c->na_ev) == hipSuccess)
      c->na_inflight = false;
    else
      return true;
  }
  for (Sub &s : c->subs) {
    if (!s.inflight) continue;
    if ((s.done_seq && __atomic_load_n(sub_done_word(c, s), __ATOMIC_ACQUIRE) == s.done_seq) ||
        hipEventQuery(s.ev) == hipSuccess)
      s.inflight = false;
    else
      return true;
  }
  return false;
}

hipError_t sync_event(hipEvent_t e) {
  // A fence usually waits for a few microseconds of GPU work: poll first
  // (hipEventSynchronize may sleep and wake tens of microseconds late), then
  // block, so a long wait does not burn a core.
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t q = hipEventQuery(e);
    if (q != hipErrorNotReady) return q;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(200)) break;
  }
  return hipEventSynchronize(e);
}

bool wait_done(const uint64_t *w, uint64_t seq) {
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t k = 0;; k++) {
    if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == seq) return true;
    if ((k & 63) == 63 && std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(200))
      return false;
  }
}

bool writes_device_only(hicr_ctx c, const hicr_desc *d, uint64_t n) {
  for (uint64_t i = 0; i < n; i++)
    if (c->slots[d[i].dst_slot].space != HICR_MEM_HBM) return false;
  return true;
}

// A submission that raises a done word has ended once the word holds its
// value (the event completes ~5 us later on gfx950 with ROCm 7); otherwise,
// or if the word is late, the event decides.
int wait_sub(hicr_ctx c, Sub &s) {
  if (!s.inflight) return HICR_OK;
  if (s.done_seq && wait_done(sub_done_word(c, s), s.done_seq)) {
    s.inflight = false;
    return HICR_OK;
  }
  hipError_t e = sync_event(s.ev);
  s.inflight = false;
  if (e != hipSuccess) return hip_fail(c, e, "waiting for a batch");
  return HICR_OK;
}

int wait_all(hicr_ctx c) {
  int rc = HICR_OK;
  for (Sub &s : c->subs) {
    int r = wait_sub(c, s);
    if (r != HICR_OK) rc = r;
  }
  if (c->na_inflight) {
    hipError_t e = sync_event(c->na_ev);
    c->na_inflight = false;
    c->na_up_pending = false;  // the upload precedes the launches on one stream
    if (e != hipSuccess) rc = hip_fail(c, e, "waiting for a no-allocation batch");
  }
  int r = wait_extra(c);
  if (r != HICR_OK) rc = r;
  r = wait_plans(c);
  if (r != HICR_OK) rc = r;
  return rc;
}

static int ensure_capacity(hicr_ctx c, Sub &s, uint64_t n) {
  if (n <= s.cap) return HICR_OK;
  uint64_t cap = std::max<uint64_t>(n, std::max<uint64_t>(2 * s.cap, 4096));
  if (s.h) (void)hipHostFree(s.h);
  if (s.d) (void)hipFree(s.d);
  s.h = nullptr;
  s.d = nullptr;
  s.cap = 0;
  hipError_t e = hipHostMalloc(&s.h, cap * 32, hipHostMallocDefault);
  if (e != hipSuccess) return fail(c, HICR_ENOMEM, "pinned staging of %llu requests", (unsigned long long)cap);
  e = hipMalloc(&s.d, batch_bytes(cap));
  if (e != hipSuccess) return fail(c, HICR_ENOMEM, "device batch buffer of %llu requests", (unsigned long long)cap);
  s.cap = cap;
  return HICR_OK;
}

// The counter table is allocated once, for kMaxSlots slots (16 MiB), so its
// address never changes: captured plans keep a valid pointer to it.
static int alloc_counters(hicr_ctx c) {
  hipError_t e = hipMalloc(&c->d_counters, (size_t)kMaxSlots * 16);
  if (e == hipSuccess) e = hipMemset(c->d_counters, 0, (size_t)kMaxSlots * 16);
  if (e != hipSuccess) return hip_fail(c, e, "allocating the counter table");
  c->counter_cap = kMaxSlots;
  return HICR_OK;
}

// Copy workgroups per CU when the caller has not fixed it.  Measured on the
// batched workload (256 CUs): with 64 KiB or 1 MiB pieces two workgroups per
// CU (eight wavefronts, each with two rounds of `unroll` 1 KiB rows in
// flight) are the fastest at either unroll, 1-2 % above one or four; 4 KiB
// pieces spend more time per piece on the search and want four.  32 KiB
// pieces at unroll 4 run 1.7 % faster with one workgroup per CU than with
// two (0.6-1 % on 64 MiB copies, aligned or not); 24 KiB pieces tie, 48 KiB
// pieces lose 0.6 %.  Pieces of 16 KiB or less get at least four from the
// latency rule in launch_copies.
int default_grid_per_cu(const DevSched &ds) {
  if (ds.chunk <= (4u << 10)) return 4;
  if (ds.chunk <= (32u << 10)) return 1;
  return 2;
}

int split_batch(hicr_ctx c, const uint64_t *hd, const uint64_t *hz, uint64_t n, const DevSched &ds,
                std::vector<Seg> &out) {
  out.clear();
  const bool lds = n <= kMaxLdsDescs;
  if (!lds) {
    // A piece spans at least 128 destination bytes except at a request's
    // ends, so a request has at most size / 128 + 2 pieces.  When that bound
    // keeps the batch under 2^31 pieces, no per-request count is needed on
    // the host (the scan kernel counts): launches split by request count
    // only, and `pieces` holds the lower bound, one per request.
    uint64_t bytes = 0;
    for (uint64_t i = 0; i < n; i++) bytes += hz[i];
    if (bytes < (1ull << 38) && (bytes >> 7) + 2 * n < (1ull << 31)) {
      const uint64_t cap = (uint64_t)kTile * kMaxTiles;
      for (uint64_t i0 = 0; i0 < n; i0 += cap) {
        const uint64_t i1 = std::min(n, i0 + cap);
        uint64_t b = bytes;
        if (i0 > 0 || i1 < n) {
          b = 0;
          for (uint64_t i = i0; i < i1; i++) b += hz[i];
        }
        out.push_back(Seg{i0, i1, i1 - i0, b, false});
      }
      return HICR_OK;
    }
  }
  uint64_t i0 = 0;
  while (i0 < n) {
    uint64_t i1 = i0, pieces = 0, bytes = 0;
    const uint64_t cap = lds ? kMaxLdsDescs : (uint64_t)kTile * kMaxTiles;
    while (i1 < n && i1 - i0 < cap) {
      uint64_t p = piece_count(hd[i1], hz[i1], ds.chunk, ds.wgs);
      if (i1 > i0 && pieces + p >= (1ull << 31)) break;
      pieces += p;
      bytes += hz[i1];
      i1++;
    }
    if (pieces >= (1ull << 31))
      return fail(c, HICR_EINVAL, "request %llu needs more than 2^31 pieces",
                  (unsigned long long)i0);
    out.push_back(Seg{i0, i1, pieces, bytes, lds});
    i0 = i1;
  }
  return HICR_OK;
}

static DevBatch seg_batch(const uint64_t *dd, uint64_t n, const Seg &g) {
  return DevBatch{dd + g.i0, dd + n + g.i0, dd + 2 * n + g.i0, dd + 3 * n + g.i0,
                  (uint32_t)(g.i1 - g.i0)};
}

int launch_scans(hicr_ctx c, const uint64_t *dd, uint64_t n, const std::vector<Seg> &segs,
                 DevSched ds, uint32_t *tables, hipStream_t stream) {
  for (const Seg &g : segs) {
    if (g.lds) continue;
    hipError_t e = launch_scan(seg_batch(dd, n, g), ds, tables + g.i0, tables + n + g.i0, stream);
    if (e != hipSuccess) return hip_fail(c, e, "launching the scan kernel");
  }
  return HICR_OK;
}

int launch_copies(hicr_ctx c, const uint64_t *dd, uint64_t n, const std::vector<Seg> &segs,
                  DevSched ds, const uint32_t *tables, uint64_t *counters, hipStream_t stream,
                  uint64_t *done, uint64_t seq, bool *armed) {
  if (armed) *armed = false;
  const int per_cu_class = c->grid_per_cu > 0 ? c->grid_per_cu : default_grid_per_cu(ds);
  for (const Seg &g : segs) {
    // A launch over a scanned table whose pieces average under 16 KiB (a
    // halo exchange's rows) is latency-bound: four groups per CU measured
    // 1.45x faster than one at unroll 4.  (With an LDS table every group
    // re-scans the batch, so more groups cost more there.)
    int per_cu = per_cu_class;
    if (c->grid_per_cu == 0 && !g.lds &&
        (ds.chunk <= (16u << 10) || g.bytes < (g.i1 - g.i0) * (16u << 10)))
      per_cu = std::max(per_cu, 4);
    per_cu = std::min(per_cu, c->occ);
    const uint64_t cap_grid = (uint64_t)c->n_cu * (uint64_t)per_cu;
    // every wavefront of a workgroup copies its own pieces
    const uint64_t want = (g.pieces + kCopyBlock / 64 - 1) / (kCopyBlock / 64);
    const uint32_t grid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(want, 1), cap_grid);
    hipError_t e = g.lds ? launch_copy(seg_batch(dd, n, g), ds, grid, stream)
                         : launch_copy_mem(seg_batch(dd, n, g), ds, tables + g.i0,
                                           tables + n + g.i0, grid, stream);
    if (e != hipSuccess) return hip_fail(c, e, "launching the copy kernel");
  }
  if (counters && n) {
    hipError_t e = launch_count(dd + 3 * n, n, counters, stream, done, seq, armed);
    if (e != hipSuccess) return hip_fail(c, e, "launching the counter kernel");
  }
  return HICR_OK;
}

void pack_batch(hicr_ctx c, const hicr_desc *d, uint64_t n, uint64_t *h) {
  uint64_t *hd = h, *hs = h + n, *hz = h + 2 * n, *hp = h + 3 * n;
  for (uint64_t i = 0; i < n; i++) {
    hd[i] = c->slots[d[i].dst_slot].base + d[i].dst_off;
    hs[i] = c->slots[d[i].src_slot].base + d[i].src_off;
    hz[i] = d[i].size;
    hp[i] = (uint64_t)d[i].dst_slot | ((uint64_t)d[i].src_slot << 32);
  }
}

// Host threads for batches large enough that validating and packing them on
// one core would take longer than their copy (a halo exchange: 61,952
// requests, ~186 us on one core).  run(f) calls f(part) for every part in
// [0, size()), part 0 on the calling thread, and returns when all are done.
class HostPool {
 public:
  explicit HostPool(int extra) {
    try {
      for (int i = 0; i < extra; i++) th_.emplace_back([this, i] { loop(i + 1); });
    } catch (...) {
      stop();  // join the threads already started, then report the failure
      throw;
    }
  }
  ~HostPool() { stop(); }
  int size() const { return (int)th_.size() + 1; }
  void run(const std::function<void(int)> &f) {
    {
      std::lock_guard<std::mutex> g(m_);
      f_ = &f;
      left_ = (int)th_.size();
      gen_++;
    }
    cv_.notify_all();
    f(0);
    std::unique_lock<std::mutex> g(m_);
    done_.wait(g, [&] { return left_ == 0; });
    f_ = nullptr;
  }

 private:
  void stop() {
    {
      std::lock_guard<std::mutex> g(m_);
      quit_ = true;
    }
    cv_.notify_all();
    for (std::thread &t : th_)
      if (t.joinable()) t.join();
  }
  void loop(int part) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int)> *f;
      {
        std::unique_lock<std::mutex> g(m_);
        cv_.wait(g, [&] { return quit_ || gen_ != seen; });
        if (quit_) return;
        seen = gen_;
        f = f_;
      }
      (*f)(part);
      std::lock_guard<std::mutex> g(m_);
      if (--left_ == 0) done_.notify_one();
    }
  }
  std::vector<std::thread> th_;
  std::mutex m_;
  std::condition_variable cv_, done_;
  const std::function<void(int)> *f_ = nullptr;
  uint64_t gen_ = 0;
  int left_ = 0;
  bool quit_ = false;
};

void destroy_pool(hicr_ctx c) {
  delete c->pool;
  c->pool = nullptr;
}

constexpr uint64_t kPoolMin = 16384;        // requests that make a batch large
constexpr uint64_t kUploadStream = 256 << 10;  // upload bytes that go on their own stream

// Validate and pack requests [i0, i1); the index of the first rejected one
// (and its code), or i1.
static uint64_t pack_range(hicr_ctx c, const hicr_desc *d, uint64_t n, uint64_t i0, uint64_t i1,
                           uint64_t *h, int *rc_out) {
  uint64_t *hd = h, *hs = h + n, *hz = h + 2 * n, *hp = h + 3 * n;
  const Slot *sl = c->slots.data();
  for (uint64_t i = i0; i < i1; i++) {
    const hicr_desc &x = d[i];
    const int rc = check_desc(c, x);
    if (rc != HICR_OK) {
      *rc_out = rc;
      return i;
    }
    hd[i] = sl[x.dst_slot].base + x.dst_off;
    hs[i] = sl[x.src_slot].base + x.src_off;
    hz[i] = x.size;
    hp[i] = (uint64_t)x.dst_slot | ((uint64_t)x.src_slot << 32);
  }
  return i1;
}

// Validate, pack and launch n requests as one submission.
int submit(hicr_ctx c, const hicr_desc *d, uint64_t n, const hicr_sched &sched,
           hipStream_t stream, uint64_t *bad, const SubmitOpts *opt) {
  if (n == 0) return HICR_OK;
  // Choose the submission buffer (round robin; wait if still in flight).
  Sub &s = c->subs[c->next_sub];
  c->next_sub = (c->next_sub + 1) % kNumSubs;
  int rc = wait_sub(c, s);
  if (rc != HICR_OK) return rc;
  rc = ensure_capacity(c, s, n);
  if (rc != HICR_OK) return rc;
  // validate and pack in one pass (split over host threads for a large
  // batch); nothing is queued unless every request passes and the batch
  // splits into launches
  uint64_t *h = static_cast<uint64_t *>(s.h);
  uint64_t first_bad = n;
  int bad_rc = HICR_OK;
  if (n >= kPoolMin && !c->pool && !c->pool_failed) {
    // no exception crosses the C ABI: a pool that cannot start its threads
    // leaves the checks on the calling thread
    try {
      const int hw = (int)std::thread::hardware_concurrency();
      c->pool = new HostPool(std::max(0, std::min(3, hw - 1)));
    } catch (...) {
      c->pool = nullptr;
      c->pool_failed = true;
    }
  }
  if (n >= kPoolMin && c->pool && c->pool->size() > 1) {
    const int parts = c->pool->size();
    std::vector<uint64_t> pb(parts, n);
    std::vector<int> prc(parts, HICR_OK);
    c->pool->run([&](int p) {
      const uint64_t i0 = n * p / parts, i1 = n * (p + 1) / parts;
      const uint64_t b = pack_range(c, d, n, i0, i1, h, &prc[p]);
      if (b < i1) pb[p] = b;
    });
    for (int p = 0; p < parts; p++)
      if (pb[p] < first_bad) {
        first_bad = pb[p];
        bad_rc = prc[p];
      }
  } else {
    first_bad = pack_range(c, d, n, 0, n, h, &bad_rc);
  }
  if (first_bad < n) {
    if (bad) *bad = first_bad;
    return fail(c, bad_rc, "request %llu rejected", (unsigned long long)first_bad);
  }
  DevSched ds{sched.chunk_bytes, sched.wgs_per_desc, sched.unroll, 0};
  rc = split_batch(c, h, h + 2 * n, n, ds, c->segs);
  if (rc != HICR_OK) return rc;
  // a large upload runs on its own stream, so it overlaps the copies queued
  // before it; the copy stream waits for it
  hipError_t e;
  if (n * 32 >= kUploadStream) {
    e = hipMemcpyAsync(s.d, s.h, n * 32, hipMemcpyHostToDevice, c->up);
    if (e == hipSuccess) e = hipEventRecord(s.up_ev, c->up);
    if (e == hipSuccess) e = hipStreamWaitEvent(stream, s.up_ev, 0);
  } else {
    e = hipMemcpyAsync(s.d, s.h, n * 32, hipMemcpyHostToDevice, stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "uploading a batch");
  const uint64_t *dd = static_cast<const uint64_t *>(s.d);
  uint64_t *counters = (opt && opt->no_count) ? nullptr : c->d_counters;
  if (opt && opt->t0) {
    e = hipEventRecord(opt->t0, stream);
    if (e != hipSuccess) return hip_fail(c, e, "recording a timing event");
  }
  uint32_t *tables = batch_tables(s.d, n);
  // a batch small enough for one counter group that writes device memory
  // only announces its end in the buffer's done word
  uint64_t *done = nullptr, seq = 0;
  if (counters && n <= 1024 && writes_device_only(c, d, n)) {
    done = sub_done_word(c, s);
    seq = ++c->done_next;
  }
  bool armed = false;
  s.done_seq = 0;
  rc = launch_scans(c, dd, n, c->segs, ds, tables, stream);
  if (rc == HICR_OK)
    rc = launch_copies(c, dd, n, c->segs, ds, tables, counters, stream, done, seq, &armed);
  if (rc == HICR_OK && armed) s.done_seq = seq;
  if (rc == HICR_OK && opt && opt->t1) {
    e = hipEventRecord(opt->t1, stream);
    if (e != hipSuccess) rc = hip_fail(c, e, "recording a timing event");
  }
  // the staging buffer is in use from the upload on, whatever failed after it
  e = hipEventRecord(s.ev, stream);
  if (e == hipSuccess) s.inflight = true;
  if (rc != HICR_OK) return rc;
  if (e != hipSuccess) return hip_fail(c, e, "recording a batch event");
  return HICR_OK;
}

int flush_pending(hicr_ctx c) {
  if (c->pending.empty()) return HICR_OK;
  std::vector<hicr_desc> p;
  p.swap(c->pending);
  uint64_t bad = 0;
  return submit(c, p.data(), p.size(), c->def_sched, c->stream, &bad, nullptr);
}

}  // namespace hicr

// ---------------------------------------------------------------- C ABI

extern "C" {

int hicr_sched_class(uint32_t cls, hicr_sched *out) {
  return guarded([&]() -> int {
    if (!out || cls >= HICR_NUM_CLASSES) return HICR_EINVAL;
    out->chunk_bytes = kChunks[cls / 4];
    out->wgs_per_desc = kWgs[(cls / 2) % 2];
    out->unroll = kUnroll[cls % 2];
    out->mode = HICR_SCHED_FIXED;
    return HICR_OK;
  });
}

const char *hicr_strerror(int code) {
  switch (code) {
    case HICR_OK: return "ok";
    case HICR_EINVAL: return "invalid argument";
    case HICR_ERANGE: return "offset or size outside the slot";
    case HICR_EBADSLOT: return "unknown or deregistered slot";
    case HICR_EUNSUPPORTED: return "memory-space pair not supported";
    case HICR_EAGAIN: return "channel full or empty; try again";
    case HICR_ENOMEM: return "out of memory";
    case HICR_ETIMEDOUT: return "timed out";
    case HICR_EHAZARD: return "conflicting requests in one epoch";
    case HICR_EDEVICE: return "device or HIP runtime error";
    case HICR_EBUSY: return "transfers still in flight";
    default: return "unknown error";
  }
}

int hicr_last_error(hicr_ctx c, char *buf, size_t n) {
  return guarded([&]() -> int {
    if (!c || !buf || n == 0) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    snprintf(buf, n, "%s", c->err.c_str());
    return HICR_OK;
  });
}

int hicr_ctx_create(int device, void *stream, hicr_ctx *out) {
  return guarded([&]() -> int {
    if (!out) return HICR_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HICR_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return HICR_EDEVICE;
    hicr_ctx c = new (std::nothrow) hicr_ctx_s();
    if (!c) return HICR_ENOMEM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
      delete c;
      return HICR_EDEVICE;
    }
    c->n_cu = prop.multiProcessorCount;
    if (copy_occupancy(&c->occ) != 0 || c->occ < 1) c->occ = 1;
    if (stream) {
      c->stream = static_cast<hipStream_t>(stream);
      c->own_stream = false;
    } else if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return HICR_EDEVICE;
    } else {
      c->own_stream = true;
    }
    bool ok = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipHostMalloc(&c->h_read, 64, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc(&c->h_done, 64 * kNumSubs, hipHostMallocDefault) == hipSuccess;
    if (ok) std::memset(c->h_done, 0, 64 * kNumSubs);
    ok = ok && hipEventCreateWithFlags(&c->push_ev, hipEventDisableTiming) == hipSuccess;
    if (ok && (pump_occupancy(&c->pump_occ) != 0 || c->pump_occ < 1)) c->pump_occ = 1;
    ok = ok && hipStreamCreateWithFlags(&c->up, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; ok && i < kNumSubs; i++) {
      ok = hipEventCreateWithFlags(&c->subs[i].ev, hipEventDisableTiming) == hipSuccess;
      ok = ok && hipEventCreateWithFlags(&c->subs[i].up_ev, hipEventDisableTiming) == hipSuccess;
    }
    c->def_sched = hicr_sched{64u << 10, 1, 2, HICR_SCHED_FIXED};
    // what hicr_memcpy_batch_noalloc needs, set up once here: the device
    // workspace's address, pinned staging, its events, and room for its
    // launch list and error messages (so that no call of it allocates)
    ok = ok && noalloc_scratch(device, &c->na_scratch) == hipSuccess;
    ok = ok && hipHostMalloc(&c->na_h, kNoAllocMaxReqs * 32, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->na_up_ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->na_ev, hipEventDisableTiming) == hipSuccess;
    if (ok) {
      c->segs.reserve(kNoAllocSegCap);
      c->err.reserve(512);
    }
    if (!ok || alloc_counters(c) != HICR_OK) {
      hicr_ctx_destroy(c);
      return HICR_EDEVICE;
    }
    *out = c;
    return HICR_OK;
  });
}

int hicr_ctx_destroy(hicr_ctx c) {
  return guarded([&]() -> int {
    if (!c) return HICR_EINVAL;
    (void)hipSetDevice(c->device);
    wait_all(c);
    destroy_plans(c);
    destroy_extra(c);
    destroy_pump_bufs(c);
    destroy_sched(c);
    destroy_pool(c);
    for (Sub &s : c->subs) {
      if (s.h) (void)hipHostFree(s.h);
      if (s.d) (void)hipFree(s.d);
      if (s.ev) (void)hipEventDestroy(s.ev);
      if (s.up_ev) (void)hipEventDestroy(s.up_ev);
    }
    if (c->d_counters) (void)hipFree(c->d_counters);
    if (c->h_read) (void)hipHostFree(c->h_read);
    if (c->h_done) (void)hipHostFree(c->h_done);
    if (c->na_h) (void)hipHostFree(c->na_h);
    if (c->na_up_ev) (void)hipEventDestroy(c->na_up_ev);
    if (c->na_ev) (void)hipEventDestroy(c->na_ev);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    if (c->up) (void)hipStreamDestroy(c->up);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return HICR_OK;
  });
}

int hicr_ctx_set_sched(hicr_ctx c, const hicr_sched *s) {
  return guarded([&]() -> int {
    if (!c || !s) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (s->mode != HICR_SCHED_FIXED) return fail(c, HICR_EINVAL, "default schedule must be fixed");
    int rc = check_sched(c, *s);
    if (rc == HICR_OK) c->def_sched = *s;
    return rc;
  });
}

int hicr_ctx_set_copy_grid(hicr_ctx c, uint32_t wgs_per_cu) {
  return guarded([&]() -> int {
    if (!c || wgs_per_cu > 64) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    c->grid_per_cu = (int)wgs_per_cu;
    return HICR_OK;
  });
}

int hicr_ctx_set_pairs(hicr_ctx c, uint32_t pair_mask) {
  return guarded([&]() -> int {
    if (!c || (pair_mask & ~HICR_PAIRS_ALL)) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    c->pair_mask = pair_mask;
    return HICR_OK;
  });
}

int hicr_slot_register(hicr_ctx c, void *ptr, uint64_t size, uint32_t memspace, hicr_slot *out) {
  return guarded([&]() -> int {
    if (!c || !out) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    if (!ptr) return fail(c, HICR_EINVAL, "null address");
    if (size == 0) return fail(c, HICR_EINVAL, "a slot needs a non-zero size");
    if (memspace != HICR_MEM_HBM && memspace != HICR_MEM_HOST)
      return fail(c, HICR_EINVAL, "unknown memory space %u", memspace);
    if (memspace == HICR_MEM_HBM) {
      hipPointerAttribute_t attr;
      if (hipPointerGetAttributes(&attr, ptr) != hipSuccess || attr.type != hipMemoryTypeDevice ||
          attr.device != c->device) {
        (void)hipGetLastError();
        return fail(c, HICR_EINVAL, "address is not device memory of device %d", c->device);
      }
      hipDeviceptr_t base = nullptr;
      size_t alloc = 0;
      if (hipMemGetAddressRange(&base, &alloc, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, HICR_EINVAL, "address outside every device allocation");
      }
      uint64_t b = reinterpret_cast<uint64_t>(base), p = reinterpret_cast<uint64_t>(ptr);
      if (p - b > alloc || size > alloc - (p - b))
        return fail(c, HICR_ERANGE, "slot extends past the end of its allocation");
    }
    uint64_t dev_addr = reinterpret_cast<uint64_t>(ptr);
    if (memspace == HICR_MEM_HOST) {
      // pinned host memory: the device reaches it at its device-side address
      hipPointerAttribute_t attr;
      if (hipPointerGetAttributes(&attr, ptr) != hipSuccess || attr.type != hipMemoryTypeHost) {
        (void)hipGetLastError();
        return fail(c, HICR_EINVAL, "address is not pinned host memory");
      }
      void *dp = nullptr;
      if (hipHostGetDevicePointer(&dp, ptr, 0) != hipSuccess || !dp) {
        (void)hipGetLastError();
        return fail(c, HICR_EINVAL, "pinned host memory without a device address");
      }
      dev_addr = reinterpret_cast<uint64_t>(dp);
      void *last = static_cast<char *>(ptr) + (size - 1);
      void *dlast = nullptr;
      if (size > 1 && (hipHostGetDevicePointer(&dlast, last, 0) != hipSuccess ||
                       reinterpret_cast<uint64_t>(dlast) != dev_addr + (size - 1))) {
        (void)hipGetLastError();
        return fail(c, HICR_ERANGE, "slot extends past the end of its pinned allocation");
      }
    }
    if (c->slots.size() >= kMaxSlots)
      return fail(c, HICR_ENOMEM, "at most %u slots per context", kMaxSlots);
    Slot s;
    s.base = dev_addr;
    s.size = size;
    s.space = memspace;
    s.live = true;
    c->slots.push_back(s);
    *out = (hicr_slot)(c->slots.size() - 1);
    return HICR_OK;
  });
}

int hicr_slot_deregister(hicr_ctx c, hicr_slot slot) {
  return guarded([&]() -> int {
    if (!c) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (slot >= c->slots.size() || !c->slots[slot].live) return fail(c, HICR_EBADSLOT, "bad slot");
    for (const hicr_desc &d : c->pending)
      if (d.dst_slot == slot || d.src_slot == slot)
        return fail(c, HICR_EBUSY, "slot has unsubmitted transfers; fence first");
    if (c->slots[slot].plan_refs)
      return fail(c, HICR_EBUSY, "slot is used by %u plan(s)", c->slots[slot].plan_refs);
    if (c->slots[slot].dobj_refs)
      return fail(c, HICR_EBUSY, "slot holds %u published data object(s)", c->slots[slot].dobj_refs);
    (void)hipSetDevice(c->device);
    if (any_inflight(c) || extra_inflight(c) || plans_inflight(c))
      return fail(c, HICR_EBUSY, "transfers in flight; fence first");
    c->slots[slot].live = false;
    return HICR_OK;
  });
}

int hicr_slot_counters(hicr_ctx c, hicr_slot slot, uint64_t *sent, uint64_t *recv) {
  return guarded([&]() -> int {
    if (!c) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (slot >= c->slots.size() || !c->slots[slot].live) return fail(c, HICR_EBADSLOT, "bad slot");
    (void)hipSetDevice(c->device);
    hipError_t e = hipMemcpyAsync(c->h_read, c->d_counters + 2 * slot, 16, hipMemcpyDeviceToHost,
                                  c->aux);
    if (e == hipSuccess) e = hipStreamSynchronize(c->aux);
    if (e != hipSuccess) return hip_fail(c, e, "reading counters");
    if (sent) *sent = c->h_read[0];
    if (recv) *recv = c->h_read[1];
    return HICR_OK;
  });
}

int hicr_memcpy(hicr_ctx c, hicr_slot dst, uint64_t dst_off, hicr_slot src, uint64_t src_off,
                uint64_t size) {
  return guarded([&]() -> int {
    if (!c) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    hicr_desc d{dst, src, dst_off, src_off, size};
    int rc = check_desc(c, d);
    if (rc != HICR_OK) return fail(c, rc, "memcpy rejected");
    c->pending.push_back(d);
    if (c->pending.size() >= kMaxLdsDescs) {
      (void)hipSetDevice(c->device);
      return flush_pending(c);
    }
    return HICR_OK;
  });
}

int hicr_memcpy_batch(hicr_ctx c, const hicr_desc *descs, uint64_t n, const hicr_sched *s,
                      void *stream, uint64_t *bad) {
  return guarded([&]() -> int {
    if (!c || (n && !descs)) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    hicr_sched sched = s ? *s : c->def_sched;
    if (sched.mode == HICR_SCHED_TUNED || sched.mode == HICR_SCHED_LEARNED) {
      int rc = choose_sched(c, descs, n, sched.mode, &sched);
      if (rc != HICR_OK) return rc;
    } else if (sched.mode != HICR_SCHED_FIXED) {
      return fail(c, HICR_EINVAL, "unknown schedule mode %u", sched.mode);
    }
    int rc = check_sched(c, sched);
    if (rc != HICR_OK) return rc;
    rc = flush_pending(c);
    if (rc != HICR_OK) return rc;
    return submit(c, descs, n, sched,
                  stream ? static_cast<hipStream_t>(stream) : c->stream, bad, nullptr);
  });
}

int hicr_memcpy_batch_noalloc(hicr_ctx c, const hicr_desc *descs, uint64_t n, const hicr_sched *s,
                              void *stream, uint64_t *bad) {
  return guarded([&]() -> int {
    if (!c || (n && !descs)) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (n > kNoAllocMaxReqs)
      return fail(c, HICR_EINVAL, "%llu requests: the no-allocation path takes at most %llu",
                  (unsigned long long)n, (unsigned long long)kNoAllocMaxReqs);
    const hicr_sched sched = s ? *s : c->def_sched;
    if (sched.mode != HICR_SCHED_FIXED)
      return fail(c, HICR_EINVAL, "the no-allocation path takes a fixed schedule only");
    int rc = check_sched(c, sched);
    if (rc != HICR_OK) return rc;
    if (!c->na_scratch || !c->na_h) return fail(c, HICR_EDEVICE, "no device workspace");
    if (n == 0) return HICR_OK;
    (void)hipSetDevice(c->device);
    // the staging is reused: the previous call's upload must have finished
    if (c->na_up_pending) {
      hipError_t e = hipEventSynchronize(c->na_up_ev);
      if (e != hipSuccess) return hip_fail(c, e, "waiting for the previous upload");
      c->na_up_pending = false;
    }
    uint64_t *h = static_cast<uint64_t *>(c->na_h);
    int bad_rc = HICR_OK;
    const uint64_t first_bad = pack_range(c, descs, n, 0, n, h, &bad_rc);
    if (first_bad < n) {
      if (bad) *bad = first_bad;
      return fail(c, bad_rc, "request %llu rejected", (unsigned long long)first_bad);
    }
    uint64_t bytes = 0;
    for (uint64_t i = 0; i < n; i++) bytes += h[2 * n + i];
    if (bytes >= kNoAllocMaxBytes)
      return fail(c, HICR_EINVAL, "%llu bytes: the no-allocation path moves less than 2^38 per call",
                  (unsigned long long)bytes);
    const DevSched ds{sched.chunk_bytes, sched.wgs_per_desc, sched.unroll, 0};
    rc = split_batch(c, h, h + 2 * n, n, ds, c->segs);
    if (rc != HICR_OK) return rc;
    const hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
    // upload, scans, copies and counters all run in order on one stream; a
    // previous call of this context on another stream must have left the
    // workspace first
    hipError_t e = hipSuccess;
    if (c->na_inflight) e = hipStreamWaitEvent(st, c->na_ev, 0);
    if (e == hipSuccess) e = hipMemcpyAsync(c->na_scratch, h, n * 32, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(c->na_up_ev, st);
    if (e != hipSuccess) return hip_fail(c, e, "uploading a batch");
    c->na_up_pending = true;
    const uint64_t *dd = static_cast<const uint64_t *>(c->na_scratch);
    uint32_t *tables = batch_tables(c->na_scratch, n);
    rc = launch_scans(c, dd, n, c->segs, ds, tables, st);
    if (rc == HICR_OK) rc = launch_copies(c, dd, n, c->segs, ds, tables, c->d_counters, st);
    e = hipEventRecord(c->na_ev, st);
    if (e == hipSuccess) c->na_inflight = true;
    if (rc != HICR_OK) return rc;
    if (e != hipSuccess) return hip_fail(c, e, "recording a batch event");
    return HICR_OK;
  });
}

int hicr_fence(hicr_ctx c) {
  return guarded([&]() -> int {
    if (!c) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    int rc = flush_pending(c);
    int r2 = wait_all(c);
    return rc != HICR_OK ? rc : r2;
  });
}

int hicr_fence_slot(hicr_ctx c, hicr_slot slot, uint64_t exp_sent, uint64_t exp_recv,
                    uint64_t timeout_ns) {
  return guarded([&]() -> int {
    if (!c) return HICR_EINVAL;
    {
      std::lock_guard<std::mutex> g(c->mu);
      if (slot >= c->slots.size() || !c->slots[slot].live) return fail(c, HICR_EBADSLOT, "bad slot");
      (void)hipSetDevice(c->device);
      int rc = flush_pending(c);
      if (rc != HICR_OK) return rc;
    }
    auto t0 = std::chrono::steady_clock::now();
    for (;;) {
      bool busy;
      {
        std::lock_guard<std::mutex> g(c->mu);
        busy = any_inflight(c) || extra_inflight(c) || plans_inflight(c);
      }
      uint64_t s = 0, r = 0;
      int rc = hicr_slot_counters(c, slot, &s, &r);
      if (rc != HICR_OK) return rc;
      if (s >= exp_sent && r >= exp_recv) return HICR_OK;
      if (!busy) return fail(c, HICR_ETIMEDOUT, "expected counts cannot be reached");
      auto dt = std::chrono::duration_cast<std::chrono::nanoseconds>(
                    std::chrono::steady_clock::now() - t0).count();
      if ((uint64_t)dt >= timeout_ns) return fail(c, HICR_ETIMEDOUT, "fence_slot timed out");
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  });
}

}  // extern "C"
