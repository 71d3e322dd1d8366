// serve.cpp -- a continuous-batching request server on one context.
//
// Requests (memcpy batches or channel bursts) arrive over time.  The server
// admits them in arrival order as soon as their destination buffers fit in
// an HBM arena (the budget), fuses every request admitted since the last
// launch into one copy launch and one pump launch, and keeps up to `streams`
// launches in flight so new work overlaps work already on the GPU.  When a
// launch completes, its requests are timestamped, handed to the caller's
// callback (while their results are still in the arena) and their arena
// space is released for the requests still waiting.
#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <set>
#include <thread>
#include <vector>

#include "runtime.h"

using namespace hicr;

namespace {

// First-fit allocator over [0, size) with coalescing free ranges.
class Arena {
 public:
  explicit Arena(uint64_t size) { free_[0] = size; }
  bool alloc(uint64_t n, uint64_t *off) {
    n = round(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const uint64_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += n;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    n = round(n);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  static uint64_t round(uint64_t n) { return ((n ? n : 1) + 255) & ~(uint64_t)255; }
  uint64_t peak() const { return peak_; }

 private:
  uint64_t used_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

struct Launch {
  hipEvent_t ev = nullptr;
  bool pump = false;
  Extra x;
  std::vector<uint64_t> reqs;
  std::vector<hicr_channel> chans;  // channels a pump launch drives
};

}  // namespace

extern "C" {

int hicr_serve(hicr_ctx c, const hicr_request *rq, uint64_t n, const hicr_serve_cfg *cfg,
               hicr_serve_stats *stats) {
  return guarded([&]() -> int {
    if (!c || !cfg || (n && !rq)) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    if (cfg->streams < 1 || cfg->streams > (uint32_t)kNumSubs)
      return fail(c, HICR_EINVAL, "streams must be 1..%d", kNumSubs);
    if (cfg->max_batch_reqs < 1) return fail(c, HICR_EINVAL, "max_batch_reqs must be >= 1");
    if (cfg->arena >= c->slots.size() || !c->slots[cfg->arena].live ||
        c->slots[cfg->arena].space != HICR_MEM_HBM)
      return fail(c, HICR_EBADSLOT, "arena slot");
    if (cfg->src >= c->slots.size() || !c->slots[cfg->src].live ||
        c->slots[cfg->src].space != HICR_MEM_HBM)
      return fail(c, HICR_EBADSLOT, "source slot");
    const Slot arena_slot = c->slots[cfg->arena], src_slot = c->slots[cfg->src];
    // validate every request up front: a request that can never run would stall the queue
    for (uint64_t r = 0; r < n; r++) {
      const hicr_request &q = rq[r];
      if (r && q.arrival_ns < rq[r - 1].arrival_ns)
        return fail(c, HICR_EINVAL, "request %llu arrives before its predecessor", (unsigned long long)r);
      if (Arena::round(q.hbm_bytes) > arena_slot.size)
        return fail(c, HICR_ERANGE, "request %llu needs more than the arena", (unsigned long long)r);
      if (q.kind == HICR_REQ_COPY) {
        if (!cfg->descs || q.first > cfg->n_descs || q.count > cfg->n_descs - q.first)
          return fail(c, HICR_ERANGE, "request %llu: descriptors", (unsigned long long)r);
        for (uint64_t i = q.first; i < q.first + q.count; i++) {
          const hicr_desc &d = cfg->descs[i];
          if (d.dst_off > q.hbm_bytes || d.size > q.hbm_bytes - d.dst_off ||
              d.src_off > src_slot.size || d.size > src_slot.size - d.src_off)
            return fail(c, HICR_ERANGE, "request %llu descriptor %llu out of range",
                        (unsigned long long)r, (unsigned long long)(i - q.first));
        }
      } else if (q.kind == HICR_REQ_BURST) {
        if (q.channel >= cfg->n_channels || !cfg->channels)
          return fail(c, HICR_EINVAL, "request %llu: channel", (unsigned long long)r);
        if (!cfg->msg_src_off || !cfg->msg_size || q.first > cfg->n_msgs ||
            q.count > cfg->n_msgs - q.first)
          return fail(c, HICR_ERANGE, "request %llu: messages", (unsigned long long)r);
        uint64_t tot = 0;
        const uint64_t lim = channel_payload_limit(cfg->channels[q.channel]);
        for (uint64_t i = q.first; i < q.first + q.count; i++) {
          if (cfg->msg_size[i] > lim)
            return fail(c, HICR_EINVAL, "request %llu: message larger than the ring", (unsigned long long)r);
          tot += cfg->msg_size[i];
        }
        if (tot > q.hbm_bytes)
          return fail(c, HICR_ERANGE, "request %llu: output larger than hbm_bytes", (unsigned long long)r);
      } else {
        return fail(c, HICR_EINVAL, "request %llu: kind", (unsigned long long)r);
      }
    }
    const hicr_sched base = cfg->sched_or_null ? *cfg->sched_or_null : c->def_sched;
    if (base.mode > HICR_SCHED_LEARNED) return fail(c, HICR_EINVAL, "schedule mode");
    if (base.mode == HICR_SCHED_FIXED && check_sched(c, base) != HICR_OK) return HICR_EINVAL;
    int rc = flush_pending(c);
    if (rc == HICR_OK) rc = wait_all(c);
    if (rc != HICR_OK) return rc;

    std::vector<hipStream_t> streams(cfg->streams);
    for (auto &s : streams)
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return fail(c, HICR_EDEVICE, "serving streams");
    Arena arena(arena_slot.size);
    std::vector<uint64_t> alloc_off(n, 0);
    std::deque<uint64_t> waiting;
    std::vector<Launch> inflight;
    // A channel's ring has one producer and one consumer: a burst waits while
    // a pump launch still in flight drives its channel.
    std::set<hicr_channel> busy;
    uint64_t next = 0, done = 0, n_copy = 0, n_pump = 0, max_reqs = 0;
    const auto t0 = std::chrono::steady_clock::now();
    auto now_ns = [&]() {
      return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
                 std::chrono::steady_clock::now() - t0).count();
    };
    uint32_t next_stream = 0;
    std::vector<hicr_desc> dbuf;
    std::vector<PumpStream> pbuf;
    std::vector<uint64_t> moff, msz;
    while (done < n && rc == HICR_OK) {
      bool progress = false;
      uint64_t t = now_ns();
      while (next < n && rq[next].arrival_ns <= t) waiting.push_back(next++);
      // completions
      for (size_t k = 0; k < inflight.size();) {
        Launch &L = inflight[k];
        const hipError_t q = hipEventQuery(L.ev);
        if (q == hipErrorNotReady) {
          k++;
          continue;
        }
        if (q != hipSuccess) {
          rc = hip_fail(c, q, "serving launch");
          break;
        }
        const uint64_t tc = now_ns();
        if (L.pump) {
          int r = pump_finish(c, L.x);
          if (r != HICR_OK) rc = r;
          for (hicr_channel ch : L.chans) busy.erase(ch);
        } else {
          (void)hipEventDestroy(L.ev);
        }
        for (uint64_t r : L.reqs) {
          if (cfg->done_ns) cfg->done_ns[r] = tc;
          if (cfg->on_complete) cfg->on_complete(cfg->user, r, alloc_off[r]);
          arena.release(alloc_off[r], rq[r].hbm_bytes);
          done++;
        }
        inflight.erase(inflight.begin() + k);
        progress = true;
      }
      if (rc != HICR_OK) break;
      // admission (arrival order) and one fused launch of each kind
      if (inflight.size() + 2 <= streams.size() + 1 && !waiting.empty()) {
        dbuf.clear();
        pbuf.clear();
        moff.clear();
        msz.clear();
        std::vector<uint64_t> copy_reqs, burst_reqs;
        std::vector<hicr_channel> used;
        while (!waiting.empty() && copy_reqs.size() + burst_reqs.size() < cfg->max_batch_reqs) {
          const uint64_t r = waiting.front();
          const hicr_request &q = rq[r];
          if (q.kind == HICR_REQ_BURST &&
              (busy.count(cfg->channels[q.channel]) ||
               std::find(used.begin(), used.end(), cfg->channels[q.channel]) != used.end()))
            break;  // one burst per channel in flight; a later launch takes it
          uint64_t off;
          if (!arena.alloc(q.hbm_bytes, &off)) break;  // wait until memory frees up
          alloc_off[r] = off;
          if (cfg->admit_ns) cfg->admit_ns[r] = t;
          waiting.pop_front();
          if (q.kind == HICR_REQ_COPY) {
            for (uint64_t i = q.first; i < q.first + q.count; i++) {
              hicr_desc d = cfg->descs[i];
              d.dst_slot = cfg->arena;
              d.dst_off += off;
              d.src_slot = cfg->src;
              dbuf.push_back(d);
            }
            copy_reqs.push_back(r);
          } else {
            PumpStream ps;
            ps.channel = cfg->channels[q.channel];
            ps.producer = 0;
            ps.src_base = src_slot.base;
            ps.src_size = src_slot.size;
            ps.out_base = arena_slot.base + off;
            ps.out_size = q.hbm_bytes;
            ps.first_msg = moff.size();
            ps.n_msgs = q.count;
            for (uint64_t i = q.first; i < q.first + q.count; i++) {
              moff.push_back(cfg->msg_src_off[i]);
              msz.push_back(cfg->msg_size[i]);
            }
            pbuf.push_back(ps);
            used.push_back(ps.channel);
            burst_reqs.push_back(r);
          }
        }
        if (!copy_reqs.empty()) {
          hipStream_t s = streams[next_stream++ % streams.size()];
          uint64_t bad = 0;
          Launch L;
          hicr_sched sched = base;
          if (base.mode != HICR_SCHED_FIXED)
            rc = choose_sched(c, dbuf.data(), dbuf.size(), base.mode, &sched);
          if (rc == HICR_OK) rc = submit(c, dbuf.data(), dbuf.size(), sched, s, &bad, nullptr);
          if (rc == HICR_OK && hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) != hipSuccess)
            rc = fail(c, HICR_EDEVICE, "serving event");
          if (rc == HICR_OK && hipEventRecord(L.ev, s) != hipSuccess)
            rc = fail(c, HICR_EDEVICE, "serving event");
          if (rc != HICR_OK) break;
          L.reqs = copy_reqs;
          inflight.push_back(L);
          n_copy++;
        }
        if (!burst_reqs.empty()) {
          hipStream_t s = streams[next_stream++ % streams.size()];
          Launch L;
          L.pump = true;
          rc = pump_launch(c, pbuf, moff.data(), msz.data(), moff.size(), nullptr, nullptr, 0, s,
                           &L.x);
          if (rc != HICR_OK) break;
          L.ev = L.x.ev;
          L.reqs = burst_reqs;
          L.chans = used;
          busy.insert(used.begin(), used.end());
          inflight.push_back(L);
          n_pump++;
        }
        uint64_t in_reqs = 0;
        for (const Launch &L : inflight) in_reqs += L.reqs.size();
        max_reqs = std::max(max_reqs, in_reqs);
        progress = progress || !copy_reqs.empty() || !burst_reqs.empty();
      }
      if (!progress) std::this_thread::yield();
    }
    // drain (also after an error), then release the streams
    for (Launch &L : inflight) {
      (void)hipEventSynchronize(L.ev);
      if (L.pump)
        pump_finish(c, L.x);
      else
        (void)hipEventDestroy(L.ev);
    }
    int r2 = wait_all(c);
    if (rc == HICR_OK) rc = r2;
    for (auto &s : streams) (void)hipStreamDestroy(s);
    if (stats) {
      stats->completed = done;
      stats->peak_arena_bytes = arena.peak();
      stats->copy_launches = n_copy;
      stats->pump_launches = n_pump;
      stats->max_inflight_requests = max_reqs;
      stats->wall_ns = now_ns();
    }
    return rc;
  });
}

}  // extern "C"
