// runtime.h -- the host context shared by the runtime's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hicr.h"
#include "internal.h"

struct hicr_channel_s;
struct hicr_plan_s;

namespace hicr {

struct Slot {
  uint64_t base = 0;
  uint64_t size = 0;
  uint32_t space = 0;
  uint32_t plan_refs = 0;  // plans whose requests name this slot
  uint32_t dobj_refs = 0;  // published data objects inside this slot
  bool live = false;
};

// One submission buffer: pinned staging, its device copy, the event that
// marks the end of the submission, and the value its counter kernel stores
// to the buffer's word of the context's done array when it ends.
struct Sub {
  void *h = nullptr;
  void *d = nullptr;
  uint64_t cap = 0;
  hipEvent_t ev = nullptr;     // end of the submission's last launch
  hipEvent_t up_ev = nullptr;  // end of its upload, when that ran on the upload stream
  bool inflight = false;
  uint64_t done_seq = 0;       // 0: the submission raises no done word
};

class HostPool;  // host threads that validate and pack large batches (runtime.cpp)

// One copy launch of a batch: requests [i0, i1) with `bytes` bytes and
// `pieces` pieces (exact on the LDS path, at least that many on the table
// path); `lds` when every workgroup scans the piece table into LDS itself,
// otherwise the launch reads the tables that scan_kernel wrote.
struct Seg {
  uint64_t i0, i1, pieces, bytes;
  bool lds;
};

// Extra controls of one submission (autotuner).
struct SubmitOpts {
  bool no_count = false;     // do not raise slot counters
  hipEvent_t t0 = nullptr;   // recorded just before the first scan or copy launch
  hipEvent_t t1 = nullptr;   // recorded just after the last copy launch
};

constexpr int kNumSubs = 4;
constexpr uint32_t kMaxSlots = 1u << 20;  // slots per context (fixed counter table)

struct SchedState;  // autotuned table and device-resident network (sched.cpp)

// Asynchronous work other than copy submissions (channel pushes, pumps):
// its event, and buffers to free once it has completed.
// Staging (pinned) and device buffers of a pump launch, reused by later
// launches once the pump has finished: allocating and freeing them per call
// cost ~1 ms, and hipFree waits for the device.
struct PumpBuf {
  void *h = nullptr, *d = nullptr;
  uint64_t h_cap = 0, d_cap = 0;
};

// A pump launch whose completion has not been observed yet: what later
// launches need to stay co-resident with it and off its rings.
struct PumpLive {
  hipEvent_t ev = nullptr;
  hipStream_t stream = nullptr;
  uint64_t wgs = 0;
  std::vector<struct ::hicr_channel_s *> chans;
};

struct Extra {
  hipEvent_t ev = nullptr;
  void *d_buf = nullptr;
  void *h_buf = nullptr;
  uint64_t h_cap = 0, d_cap = 0;  // sizes of h_buf and d_buf
  bool pump = false;
  uint32_t *abort_word = nullptr;
  std::vector<struct ::hicr_channel_s *> chans;
};

}  // namespace hicr

struct hicr_ctx_s {
  std::mutex mu;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t aux = nullptr;  // counter reads, never waits on `stream`
  hipStream_t up = nullptr;   // uploads of large batches, overlapping earlier copies
  hicr::HostPool *pool = nullptr;  // created at the first large submission
  bool pool_failed = false;        // its threads could not be started
  int n_cu = 1;
  int occ = 1;       // copy workgroups per CU that fit
  int grid_per_cu = 0;  // copy workgroups per CU launched (0: per-schedule default)
  uint32_t pair_mask = HICR_PAIRS_ALL;  // memory-space pairs memcpy accepts
  std::vector<hicr::Slot> slots;
  uint64_t *d_counters = nullptr;  // [slot] = {sent, recv}
  uint32_t counter_cap = 0;
  uint64_t *h_read = nullptr;  // pinned read-back buffer
  hicr::Sub subs[hicr::kNumSubs];
  int next_sub = 0;
  // pinned words that one-group counter launches raise when a submission
  // ends (word 8 i for subs[i], one 64-byte line each), and the last value
  // handed out
  uint64_t *h_done = nullptr;
  uint64_t done_next = 0;
  // hicr_memcpy_batch_noalloc: this device's fixed workspace, pinned staging
  // allocated with the context, and the events of the last such submission
  void *na_scratch = nullptr;
  void *na_h = nullptr;
  hipEvent_t na_up_ev = nullptr;  // end of its upload (the staging is free again)
  hipEvent_t na_ev = nullptr;     // end of its last launch
  bool na_up_pending = false;
  bool na_inflight = false;
  std::vector<hicr::Seg> segs;  // launches of the submission being queued
  std::vector<hicr_desc> pending;
  hicr_sched def_sched{};
  hicr::SchedState *sched = nullptr;
  std::vector<struct hicr_channel_s *> channels;
  std::vector<struct hicr_plan_s *> plans;
  std::map<uint64_t, hicr_dobj_handle> dobjs;  // published data objects by id
  uint64_t next_dobj_id = 1;
  std::vector<hicr::Extra> extra;
  std::vector<hicr::PumpBuf> pump_free;  // finished pumps' buffers, for reuse
  std::vector<hicr::PumpLive> pump_live;  // pumps launched and not yet finished
  int pump_occ = 0;  // pump workgroups per CU
  hipEvent_t push_ev = nullptr;  // last host-API channel push or network step
  bool push_pending = false;
  std::mutex abort_mu;  // guards abort_words; never held while waiting on the GPU
  std::vector<uint32_t *> abort_words;  // running pumps' pinned abort words
  std::string err;
};

namespace hicr {

int fail(hicr_ctx c, int code, const char *fmt, ...);
int hip_fail(hicr_ctx c, hipError_t e, const char *what);
int check_desc(hicr_ctx c, const hicr_desc &d);
int check_sched(hicr_ctx c, const hicr_sched &s);
bool any_inflight(hicr_ctx c);
// Wait for an event: poll briefly, then block.
hipError_t sync_event(hipEvent_t e);
// Poll a done word (pinned host memory a counter kernel stores to) for up
// to 200 us; true once it holds seq.
bool wait_done(const uint64_t *w, uint64_t seq);
// Whether every request of a batch writes device memory (HBM slots): only
// then may a done word stand for the end of the batch, since the runtime's
// completion signal is what makes bytes written to host memory visible.
bool writes_device_only(hicr_ctx c, const hicr_desc *d, uint64_t n);
int wait_all(hicr_ctx c);
int submit(hicr_ctx c, const hicr_desc *d, uint64_t n, const hicr_sched &sched,
           hipStream_t stream, uint64_t *bad, const SubmitOpts *opt);
int flush_pending(hicr_ctx c);
// Resolve requests to the structure of arrays {dst, src, size, slot pair}.
void pack_batch(hicr_ctx c, const hicr_desc *d, uint64_t n, uint64_t *h);
// Split an n-request batch into copy launches (hd/hz: host copies of dst and
// size): one LDS-scanned launch up to kMaxLdsDescs requests, otherwise
// launches over a scanned table of at most kTile * kMaxTiles requests; every
// launch under 2^31 pieces.
int split_batch(hicr_ctx c, const uint64_t *hd, const uint64_t *hz, uint64_t n, const DevSched &ds,
                std::vector<Seg> &out);
// Queue the scan kernel for every launch that reads a table (tables: the
// batch_tables() region beside the uploaded batch dd).
int launch_scans(hicr_ctx c, const uint64_t *dd, uint64_t n, const std::vector<Seg> &segs,
                 DevSched ds, uint32_t *tables, hipStream_t stream);
// Queue the copy launches, then (counters != null) the counter kernel; with
// done != null a one-group counter launch ends by storing seq to *done, and
// *armed says whether it will.
int launch_copies(hicr_ctx c, const uint64_t *dd, uint64_t n, const std::vector<Seg> &segs,
                  DevSched ds, const uint32_t *tables, uint64_t *counters, hipStream_t stream,
                  uint64_t *done = nullptr, uint64_t seq = 0, bool *armed = nullptr);
// Bytes of device memory an uploaded batch of n requests takes: the packed
// requests (32 B each), then the piece tables: per-request prefixes (4 B
// each) and tile totals (a launch over requests [i0, i1) keeps its tiles at
// entry i0 of an n-entry region; it has fewer tiles than requests).
inline uint64_t batch_bytes(uint64_t n) { return n * 40; }
inline uint32_t *batch_tables(void *d, uint64_t n) {
  return reinterpret_cast<uint32_t *>(static_cast<char *>(d) + n * 32);
}

// Persistent batch plans (plan.cpp).
int wait_plans(hicr_ctx c);
bool plans_inflight(hicr_ctx c);
void destroy_plans(hicr_ctx c);

// Schedule selection (sched.cpp): the class for a batch under mode TUNED
// (nearest tuned-table entry) or LEARNED (the network: on the host, in the
// device kernels' arithmetic, per submission; by the device forward kernel
// when on_device, as for a plan's one-time choice); the context default when
// neither has data.
int choose_sched(hicr_ctx c, const hicr_desc *d, uint64_t n, uint32_t mode, hicr_sched *out,
                 bool on_device = false);
void destroy_sched(hicr_ctx c);

// Channel pushes and pumps (channel.cpp).
struct PumpStream {
  struct ::hicr_channel_s *channel;
  uint32_t producer;
  uint64_t src_base, src_size, out_base, out_size;
  uint64_t first_msg, n_msgs;
};
// msg_off/msg_size: host arrays, or (dev_tables) device arrays the kernel
// reads in place and checks itself.
int pump_launch(hicr_ctx c, const std::vector<PumpStream> &st, const uint64_t *msg_off,
                const uint64_t *msg_size, uint64_t n_msgs, uint32_t *trace_dev, uint64_t *ts_dev,
                uint64_t timeout_ns, hipStream_t s, Extra *xout, bool dev_tables = false);
int pump_finish(hicr_ctx c, Extra &x);
void destroy_pump_bufs(hicr_ctx c);
uint64_t channel_payload_limit(struct ::hicr_channel_s *ch);
int wait_extra(hicr_ctx c);
bool extra_inflight(hicr_ctx c);
void destroy_extra(hicr_ctx c);

// Every C entry point runs its body through guarded(): the ABI never throws.
// The only exceptions host code here can raise come from allocation (a
// container growing, new, a thread that cannot start), so each becomes
// HICR_ENOMEM; locks taken in the body are released on the way out.
template <class F>
inline int guarded(F &&body) noexcept {
  try {
    return body();
  } catch (...) {
    return HICR_ENOMEM;
  }
}

}  // namespace hicr
