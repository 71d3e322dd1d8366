// plan.cpp -- persistent memcpy batches replayed from a HIP graph.
//
// A plan is a batch of memcpy requests (HiCR Sec. 3.1.4) that a caller
// repeats unchanged.  Validation, address resolution, the upload, the split
// into copy launches and (for batches of more than 4,096 requests) the scan
// of the piece table happen once.  A replay queues the fused copy launches
// and the counter kernel again, either directly or --
// HICR_PLAN_GRAPH -- as one hipGraphLaunch of those launches captured from a
// private stream at creation.  The graph holds kernel nodes only; nothing in
// it needs clearing between replays.  (Measured on gfx950 with ROCm 7: a
// graph of two or five kernel nodes launches slower than the same kernels
// queued directly, so direct replay is the default.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "runtime.h"

using namespace hicr;

struct hicr_plan_s {
  hicr_ctx c = nullptr;
  uint64_t n = 0;
  void *d = nullptr;          // device SoA {dst, src, size, slot pair} + piece tables, 40 B per request
  std::vector<Seg> segs;      // copy launches of one replay
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;  // HICR_PLAN_GRAPH
  DevSched ds{};
  hipEvent_t ev = nullptr;    // end of the last replay
  hipStream_t last = nullptr; // stream of the last replay
  bool launched = false;
  std::vector<hicr_slot> slots;  // distinct slots the requests name
  // direct replays of a plan that writes device memory only and has one
  // counter group: the pinned word their counter kernel stores the replay's
  // number to, the number of the last replay, and whether it will be stored
  uint64_t *h_done = nullptr;
  uint64_t done_seq = 0;
  bool done_armed = false;
};

namespace {

void free_plan(hicr_plan p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->ev) (void)hipEventDestroy(p->ev);
  if (p->d) (void)hipFree(p->d);
  if (p->h_done) (void)hipHostFree(p->h_done);
  for (hicr_slot s : p->slots) p->c->slots[s].plan_refs--;
  delete p;
}

int wait_plan(hicr_ctx c, hicr_plan p) {
  if (!p->launched) return HICR_OK;
  if (p->done_armed && wait_done(p->h_done, p->done_seq)) {
    p->launched = false;
    return HICR_OK;
  }
  hipError_t e = sync_event(p->ev);
  p->launched = false;
  return e == hipSuccess ? HICR_OK : hip_fail(c, e, "waiting for a plan replay");
}

}  // namespace

namespace hicr {

int wait_plans(hicr_ctx c) {
  int rc = HICR_OK;
  for (hicr_plan p : c->plans) {
    int r = wait_plan(c, p);
    if (r != HICR_OK) rc = r;
  }
  return rc;
}

bool plans_inflight(hicr_ctx c) {
  for (hicr_plan p : c->plans) {
    if (!p->launched) continue;
    if ((p->done_armed && __atomic_load_n(p->h_done, __ATOMIC_ACQUIRE) == p->done_seq) ||
        hipEventQuery(p->ev) == hipSuccess)
      p->launched = false;
    else
      return true;
  }
  return false;
}

void destroy_plans(hicr_ctx c) {
  for (hicr_plan p : c->plans) {
    (void)wait_plan(c, p);
    free_plan(p);
  }
  c->plans.clear();
}

}  // namespace hicr

extern "C" {

int hicr_plan_create(hicr_ctx c, const hicr_desc *d, uint64_t n, const hicr_sched *s,
                     uint32_t flags, hicr_plan *out, uint64_t *bad) {
  return guarded([&]() -> int {
    if (!c || !out || (n && !d) || (flags & ~HICR_PLAN_GRAPH)) return HICR_EINVAL;
    *out = nullptr;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    for (uint64_t i = 0; i < n; i++) {
      int rc = check_desc(c, d[i]);
      if (rc != HICR_OK) {
        if (bad) *bad = i;
        return fail(c, rc, "plan request %llu rejected", (unsigned long long)i);
      }
    }
    hicr_sched sched = s ? *s : c->def_sched;
    if (sched.mode == HICR_SCHED_TUNED || sched.mode == HICR_SCHED_LEARNED) {
      // resolved once, the network's class by the device forward kernel:
      // every replay uses the class chosen now
      int rc = choose_sched(c, d, n, sched.mode, &sched, true);
      if (rc != HICR_OK) return rc;
    } else if (sched.mode != HICR_SCHED_FIXED) {
      return fail(c, HICR_EINVAL, "unknown schedule mode %u", sched.mode);
    }
    int rc = check_sched(c, sched);
    if (rc != HICR_OK) return rc;

    hicr_plan p = new (std::nothrow) hicr_plan_s();
    if (!p) return HICR_ENOMEM;
    p->c = c;
    p->n = n;
    std::vector<hicr_slot> sl;
    sl.reserve(2 * n);
    for (uint64_t i = 0; i < n; i++) {
      sl.push_back(d[i].dst_slot);
      sl.push_back(d[i].src_slot);
    }
    std::sort(sl.begin(), sl.end());
    sl.erase(std::unique(sl.begin(), sl.end()), sl.end());
    for (hicr_slot x : sl) c->slots[x].plan_refs++;
    p->slots = sl;

    std::vector<uint64_t> h(4 * std::max<uint64_t>(n, 1));
    pack_batch(c, d, n, h.data());
    DevSched ds{sched.chunk_bytes, sched.wgs_per_desc, sched.unroll, 0};
    p->ds = ds;
    rc = split_batch(c, h.data(), h.data() + 2 * n, n, ds, p->segs);
    if (rc != HICR_OK) {
      free_plan(p);
      return rc;
    }
    hipStream_t cs = nullptr;
    hipError_t e = hipEventCreateWithFlags(&p->ev, hipEventDisableTiming);
    if (e == hipSuccess && n && n <= 1024 && !(flags & HICR_PLAN_GRAPH) &&
        writes_device_only(c, d, n)) {
      e = hipHostMalloc(&p->h_done, 64, hipHostMallocDefault);
      if (e == hipSuccess) *p->h_done = 0;
    }
    if (e == hipSuccess && n) e = hipMalloc(&p->d, batch_bytes(n));
    if (e == hipSuccess && n) e = hipMemcpy(p->d, h.data(), n * 32, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
      if (cs) (void)hipStreamDestroy(cs);
      free_plan(p);
      return hip_fail(c, e, "allocating a plan");
    }
    const uint64_t *dd = static_cast<const uint64_t *>(p->d);
    uint32_t *tables = n ? batch_tables(p->d, n) : nullptr;
    // the piece tables are scanned once; every replay reads them
    rc = launch_scans(c, dd, n, p->segs, ds, tables, cs);
    if (rc == HICR_OK) {
      e = hipStreamSynchronize(cs);
      if (e != hipSuccess) rc = hip_fail(c, e, "scanning a plan");
    }
    if (rc != HICR_OK) {
      (void)hipStreamDestroy(cs);
      free_plan(p);
      return rc;
    }
    if (flags & HICR_PLAN_GRAPH) {
      e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
      if (e == hipSuccess) {
        rc = launch_copies(c, dd, n, p->segs, ds, tables, c->d_counters, cs);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        p->graph = graph;
        if (rc == HICR_OK && e2 != hipSuccess) rc = hip_fail(c, e2, "capturing a plan");
        if (rc == HICR_OK) {
          e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
          if (e != hipSuccess) rc = hip_fail(c, e, "instantiating a plan");
        }
      } else {
        rc = hip_fail(c, e, "capturing a plan");
      }
    }
    (void)hipStreamDestroy(cs);
    if (rc != HICR_OK) {
      free_plan(p);
      return rc;
    }
    c->plans.push_back(p);
    *out = p;
    return HICR_OK;
  });
}

int hicr_plan_launch(hicr_plan p, void *stream) {
  return guarded([&]() -> int {
    if (!p) return HICR_EINVAL;
    hicr_ctx c = p->c;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
    hipError_t e = hipSuccess;
    if (p->launched && s != p->last) e = hipStreamWaitEvent(s, p->ev, 0);
    if (e == hipSuccess && p->exec) {
      e = hipGraphLaunch(p->exec, s);
    } else if (e == hipSuccess && p->n) {
      const uint64_t *dd = static_cast<const uint64_t *>(p->d);
      // replays are ordered (same stream, or the wait above), so the word's
      // last value is the last replay's
      const uint64_t seq = p->done_seq + 1;
      bool armed = false;
      p->done_armed = false;
      int rc = launch_copies(c, dd, p->n, p->segs, p->ds, batch_tables(p->d, p->n), c->d_counters,
                             s, p->h_done, seq, &armed);
      if (rc != HICR_OK) return rc;
      if (armed) {
        p->done_seq = seq;
        p->done_armed = true;
      }
    }
    if (e == hipSuccess) e = hipEventRecord(p->ev, s);
    if (e != hipSuccess) return hip_fail(c, e, "launching a plan");
    p->launched = true;
    p->last = s;
    return HICR_OK;
  });
}

int hicr_plan_destroy(hicr_plan p) {
  return guarded([&]() -> int {
    if (!p) return HICR_EINVAL;
    hicr_ctx c = p->c;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    int rc = wait_plan(c, p);
    c->plans.erase(std::remove(c->plans.begin(), c->plans.end(), p), c->plans.end());
    free_plan(p);
    return rc;
  });
}

}  // extern "C"
