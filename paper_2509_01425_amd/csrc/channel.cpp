// channel.cpp -- host side of the ring channels (HiCR Sec. 4.3): creation,
// the non-blocking host API (push / peek / pop / depth) and the persistent
// device pump.
//
// Host-endpoint channels keep their coordination counters in host-coherent
// pinned memory: a push enqueues push_kernel, which copies the payload into
// the HBM ring and then publishes the new message counter with a
// system-scope release; the host consumer reads that counter, and its pop
// stores the released counters that the host producer checks for room.
// Device-endpoint channels keep their counters in HBM and are driven by
// pump_kernel.
#include <algorithm>
#include <cstring>
#include <map>
#include <queue>
#include <utility>
#include <vector>

#include "chan.h"
#include "residency.h"
#include "runtime.h"

using namespace hicr;

// Offset of a pump's abort word in its pinned staging: inside the 256-byte
// head that every launch zeroes, past the 8 bytes of error words that come
// back from the device at the end.
constexpr uint64_t kAbortHostOff = 128;

struct hicr_channel_s {
  hicr_ctx ctx = nullptr;
  hicr_channel_cfg cfg{};
  uint32_t n_rings = 1;
  uint64_t P = 0, E = 0;
  uint64_t payload_base = 0, entries_base = 0;
  RingCoord *coord_host = nullptr;  // host view (host endpoints)
  RingCoord *coord_dev = nullptr;   // device view
  bool broken = false;
  // Device endpoints: messages every ring has carried in earlier pumps.
  // Pumps on one channel never overlap and always drain their messages, so
  // this is the ring's message counter when the next pump starts.
  std::vector<uint64_t> dev_msgs;
  bool user_kernels = false;  // handed to caller kernels (hicr_device.h)
  struct RingHost {
    uint64_t tm = 0, tb = 0;  // producer side: enqueued
    uint64_t hm = 0, hb = 0;  // consumer side: released
    std::vector<uint64_t> ent;
  };
  std::vector<RingHost> rh;
};

namespace {

uint64_t entry_size(uint64_t e) { return e & kEntrySizeMask; }

int check_hbm_slot(hicr_ctx c, hicr_slot s, uint64_t need, const char *what) {
  if (s >= c->slots.size() || !c->slots[s].live) return fail(c, HICR_EBADSLOT, "%s: bad slot", what);
  if (c->slots[s].space != HICR_MEM_HBM)
    return fail(c, HICR_EUNSUPPORTED, "%s: slot is not in HBM", what);
  if (c->slots[s].size < need)
    return fail(c, HICR_ERANGE, "%s: slot holds %llu bytes, needs %llu", what,
                (unsigned long long)c->slots[s].size, (unsigned long long)need);
  return HICR_OK;
}

bool registered(hicr_ctx c, hicr_channel ch) {
  return std::find(c->channels.begin(), c->channels.end(), ch) != c->channels.end();
}

// A device buffer [p, p + bytes) must lie inside one allocation of the device.
int check_dev_range(hicr_ctx c, const void *p, uint64_t bytes, const char *what) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess || attr.type != hipMemoryTypeDevice ||
      attr.device != c->device) {
    (void)hipGetLastError();
    return fail(c, HICR_EINVAL, "%s is not device memory", what);
  }
  hipDeviceptr_t base = nullptr;
  size_t alloc = 0;
  if (hipMemGetAddressRange(&base, &alloc, const_cast<void *>(p)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, HICR_EINVAL, "%s outside every allocation", what);
  }
  uint64_t b = reinterpret_cast<uint64_t>(base), q = reinterpret_cast<uint64_t>(p);
  if (q - b > alloc || bytes > alloc - (q - b))
    return fail(c, HICR_ERANGE, "%s is smaller than %llu bytes", what, (unsigned long long)bytes);
  return HICR_OK;
}

DevRing dev_ring(const hicr_channel_s *ch, uint32_t r) {
  return DevRing{ch->payload_base + r * ch->P, ch->P, ch->entries_base + r * ch->E * 8, ch->E,
                 reinterpret_cast<uint64_t>(ch->coord_dev + r)};
}

void free_channel(hicr_channel ch) {
  if (ch->cfg.endpoints == HICR_CH_HOST) {
    if (ch->coord_host) (void)hipHostFree(ch->coord_host);
  } else if (ch->coord_dev) {
    (void)hipFree(ch->coord_dev);
  }
  delete ch;
}

}  // namespace

namespace hicr {

int wait_extra(hicr_ctx c) {
  int rc = HICR_OK;
  if (c->push_pending) {
    hipError_t e = sync_event(c->push_ev);
    c->push_pending = false;
    if (e != hipSuccess) rc = hip_fail(c, e, "waiting for channel pushes");
  }
  for (Extra &x : c->extra) {
    hipError_t e = sync_event(x.ev);
    if (e != hipSuccess) rc = hip_fail(c, e, "waiting for a pump");
    int r = pump_finish(c, x);
    if (rc == HICR_OK) rc = r;
  }
  c->extra.clear();
  return rc;
}

bool extra_inflight(hicr_ctx c) {
  if (c->push_pending) {
    if (hipEventQuery(c->push_ev) == hipSuccess)
      c->push_pending = false;
    else
      return true;
  }
  for (Extra &x : c->extra)
    if (hipEventQuery(x.ev) != hipSuccess) return true;
  return false;
}

void destroy_extra(hicr_ctx c) {
  wait_extra(c);
  for (hicr_channel ch : c->channels) free_channel(ch);
  c->channels.clear();
  if (c->push_ev) (void)hipEventDestroy(c->push_ev);
  c->push_ev = nullptr;
}

}  // namespace hicr

extern "C" {

int hicr_channel_create(hicr_ctx c, const hicr_channel_cfg *cfg, hicr_channel *out) {
  return guarded([&]() -> int {
    if (!c || !cfg || !out) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    *out = nullptr;
    const hicr_channel_cfg &k = *cfg;
    if (k.kind != HICR_CH_FIXED && k.kind != HICR_CH_VAR) return fail(c, HICR_EINVAL, "bad kind");
    if (k.mode > HICR_CH_MPSC_NOLOCK) return fail(c, HICR_EINVAL, "bad mode");
    if (k.endpoints != HICR_CH_HOST && k.endpoints != HICR_CH_DEVICE)
      return fail(c, HICR_EINVAL, "bad endpoints");
    if (k.mode == HICR_CH_SPSC ? k.producers != 1
                               : (k.producers < 1 || k.producers > HICR_CH_MAX_PRODUCERS))
      return fail(c, HICR_EINVAL, "producers %u not valid for the mode", k.producers);
    uint64_t P, E;
    if (k.kind == HICR_CH_FIXED) {
      if (k.token_bytes == 0 || k.capacity == 0 || k.capacity > (1ull << 40) / k.token_bytes)
        return fail(c, HICR_EINVAL, "fixed channel needs token_bytes > 0 and capacity > 0");
      P = k.capacity * k.token_bytes;
      E = k.capacity;
    } else {
      if (k.capacity == 0 || k.entries == 0 || k.capacity > kEntrySizeMask || k.entries > (1ull << 40))
        return fail(c, HICR_EINVAL, "variable channel needs capacity > 0 and entries > 0");
      P = k.capacity;
      E = k.entries;
    }
    const uint32_t rings = k.mode == HICR_CH_MPSC_NOLOCK ? k.producers : 1;
    int rc = check_hbm_slot(c, k.payload, rings * P, "payload");
    if (rc != HICR_OK) return rc;
    rc = check_hbm_slot(c, k.entries_slot, rings * E * 8, "entries");
    if (rc != HICR_OK) return rc;
    if (c->slots[k.entries_slot].base % 8) return fail(c, HICR_EINVAL, "entries slot not 8-byte aligned");
    hicr_channel ch = new (std::nothrow) hicr_channel_s();
    if (!ch) return HICR_ENOMEM;
    ch->ctx = c;
    ch->cfg = k;
    ch->n_rings = rings;
    ch->P = P;
    ch->E = E;
    ch->payload_base = c->slots[k.payload].base;
    ch->entries_base = c->slots[k.entries_slot].base;
    const size_t bytes = sizeof(RingCoord) * rings;
    hipError_t e;
    if (k.endpoints == HICR_CH_HOST) {
      void *h = nullptr;
      e = hipHostMalloc(&h, bytes, hipHostMallocCoherent | hipHostMallocMapped);
      if (e == hipSuccess) {
        std::memset(h, 0, bytes);
        ch->coord_host = static_cast<RingCoord *>(h);
        void *d = nullptr;
        e = hipHostGetDevicePointer(&d, h, 0);
        ch->coord_dev = static_cast<RingCoord *>(d);
      }
      ch->rh.resize(rings);
      for (auto &r : ch->rh) r.ent.assign(E, 0);
    } else {
      void *d = nullptr;
      e = hipMalloc(&d, bytes);
      if (e == hipSuccess) e = hipMemset(d, 0, bytes);
      ch->coord_dev = static_cast<RingCoord *>(d);
      ch->dev_msgs.assign(rings, 0);
    }
    if (e != hipSuccess) {
      free_channel(ch);
      return fail(c, HICR_ENOMEM, "coordination counters: %s", hipGetErrorString(e));
    }
    c->channels.push_back(ch);
    *out = ch;
    return HICR_OK;
  });
}

int hicr_channel_destroy(hicr_channel ch) {
  return guarded([&]() -> int {
    if (!ch) return HICR_EINVAL;
    hicr_ctx c = ch->ctx;
    std::lock_guard<std::mutex> g(c->mu);
    if (!registered(c, ch)) return HICR_EINVAL;
    (void)hipSetDevice(c->device);
    int rc = wait_all(c);
    c->channels.erase(std::find(c->channels.begin(), c->channels.end(), ch));
    free_channel(ch);
    return rc;
  });
}

int hicr_channel_push(hicr_channel ch, uint32_t producer, hicr_slot src, uint64_t src_off,
                      uint64_t count) {
  return guarded([&]() -> int {
    if (!ch) return HICR_EINVAL;
    hicr_ctx c = ch->ctx;
    std::lock_guard<std::mutex> g(c->mu);  // the producers' exclusive access
    if (ch->cfg.endpoints != HICR_CH_HOST) return fail(c, HICR_EINVAL, "device-endpoint channel");
    if (producer >= ch->cfg.producers) return fail(c, HICR_EINVAL, "no producer %u", producer);
    const bool fixed = ch->cfg.kind == HICR_CH_FIXED;
    uint64_t bytes, n_ent, ent_bytes;
    if (fixed) {
      if (count > ch->cfg.capacity) return fail(c, HICR_EINVAL, "more tokens than the ring holds");
      bytes = count * ch->cfg.token_bytes;
      n_ent = count;
      ent_bytes = ch->cfg.token_bytes;
    } else {
      if (count > ch->P) return fail(c, HICR_EINVAL, "message larger than the ring");
      bytes = count;
      n_ent = 1;
      ent_bytes = count;
    }
    if (src >= c->slots.size() || !c->slots[src].live) return fail(c, HICR_EBADSLOT, "bad source slot");
    const Slot &ss = c->slots[src];
    if (ss.space != HICR_MEM_HBM) return fail(c, HICR_EUNSUPPORTED, "source not in HBM");
    if (src_off > ss.size || bytes > ss.size - src_off) return fail(c, HICR_ERANGE, "source range");
    const uint32_t r = ch->cfg.mode == HICR_CH_MPSC_NOLOCK ? producer : 0;
    auto &h = ch->rh[r];
    const uint64_t hm = __atomic_load_n(&ch->coord_host[r].cons.w[0], __ATOMIC_ACQUIRE);
    const uint64_t hb = __atomic_load_n(&ch->coord_host[r].cons.w[1], __ATOMIC_ACQUIRE);
    if ((h.tm - hm) + n_ent > ch->E || (h.tb - hb) + bytes > ch->P)
      return HICR_EAGAIN;  // full: the consumer has not released enough room
    if (n_ent == 0) return HICR_OK;
    (void)hipSetDevice(c->device);
    PushArgs pa;
    pa.ring = dev_ring(ch, r);
    pa.src = ss.base + src_off;
    pa.bytes = bytes;
    pa.pos = h.tb % ch->P;
    pa.first_entry = h.tm;
    pa.n_entries = (uint32_t)n_ent;
    pa.producer = producer;
    pa.entry_bytes = ent_bytes;
    pa.publish = &ch->coord_dev[r].prod.w[0];
    pa.publish_value = h.tm + n_ent;
    hipError_t e = launch_push(pa, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->push_ev, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "launching a channel push");
    c->push_pending = true;
    for (uint64_t i = 0; i < n_ent; i++)
      h.ent[(h.tm + i) % ch->E] = ent_bytes | ((uint64_t)producer << 48);
    h.tm += n_ent;
    h.tb += bytes;
    return HICR_OK;
  });
}

int hicr_channel_peek(hicr_channel ch, uint32_t ring, uint64_t i, uint64_t *payload_off,
                      uint64_t *bytes, uint32_t *producer) {
  return guarded([&]() -> int {
    if (!ch) return HICR_EINVAL;
    hicr_ctx c = ch->ctx;
    std::lock_guard<std::mutex> g(c->mu);
    if (ch->cfg.endpoints != HICR_CH_HOST) return fail(c, HICR_EINVAL, "device-endpoint channel");
    if (ring >= ch->n_rings) return fail(c, HICR_EINVAL, "no ring %u", ring);
    auto &h = ch->rh[ring];
    const uint64_t tm = __atomic_load_n(&ch->coord_host[ring].prod.w[0], __ATOMIC_ACQUIRE);
    if (i >= tm - h.hm) return HICR_EAGAIN;
    uint64_t off = h.hb;
    for (uint64_t k = 0; k < i; k++) off += entry_size(h.ent[(h.hm + k) % ch->E]);
    const uint64_t e = h.ent[(h.hm + i) % ch->E];
    if (payload_off) *payload_off = ring * ch->P + off % ch->P;
    if (bytes) *bytes = entry_size(e);
    if (producer) *producer = (uint32_t)(e >> 48);
    return HICR_OK;
  });
}

int hicr_channel_pop(hicr_channel ch, uint32_t ring, uint64_t n) {
  return guarded([&]() -> int {
    if (!ch) return HICR_EINVAL;
    hicr_ctx c = ch->ctx;
    std::lock_guard<std::mutex> g(c->mu);
    if (ch->cfg.endpoints != HICR_CH_HOST) return fail(c, HICR_EINVAL, "device-endpoint channel");
    if (ring >= ch->n_rings) return fail(c, HICR_EINVAL, "no ring %u", ring);
    auto &h = ch->rh[ring];
    const uint64_t tm = __atomic_load_n(&ch->coord_host[ring].prod.w[0], __ATOMIC_ACQUIRE);
    if (n > tm - h.hm) return HICR_EAGAIN;
    for (uint64_t k = 0; k < n; k++) h.hb += entry_size(h.ent[(h.hm + k) % ch->E]);
    h.hm += n;
    __atomic_store_n(&ch->coord_host[ring].cons.w[1], h.hb, __ATOMIC_RELEASE);
    __atomic_store_n(&ch->coord_host[ring].cons.w[0], h.hm, __ATOMIC_RELEASE);
    return HICR_OK;
  });
}

int hicr_channel_depth(hicr_channel ch, uint32_t ring, uint64_t *msgs, uint64_t *bytes) {
  return guarded([&]() -> int {
    if (!ch) return HICR_EINVAL;
    hicr_ctx c = ch->ctx;
    std::lock_guard<std::mutex> g(c->mu);
    if (ch->cfg.endpoints != HICR_CH_HOST) return fail(c, HICR_EINVAL, "device-endpoint channel");
    if (ring >= ch->n_rings) return fail(c, HICR_EINVAL, "no ring %u", ring);
    auto &h = ch->rh[ring];
    const uint64_t tm = __atomic_load_n(&ch->coord_host[ring].prod.w[0], __ATOMIC_ACQUIRE);
    uint64_t b = 0;
    for (uint64_t k = h.hm; k < tm; k++) b += entry_size(h.ent[k % ch->E]);
    if (msgs) *msgs = tm - h.hm;
    if (bytes) *bytes = b;
    return HICR_OK;
  });
}

}  // extern "C"

namespace hicr {

// Validate a pump plan whose streams carry resolved addresses, build the
// device tables and launch.  The caller holds c->mu.  On success the launch
// is described by *x (event, buffers to free, abort word, channels).
// A finished pump's buffers with room for `h_bytes` of staging and
// `d_bytes` on the device, or new ones (rounded up to a power of two, so that
// pumps of varying size settle on a few buffers).
static int take_pump_buf(hicr_ctx c, uint64_t h_bytes, uint64_t d_bytes, Extra &x) {
  for (size_t k = 0; k < c->pump_free.size(); k++) {
    const PumpBuf &b = c->pump_free[k];
    if (b.h_cap >= h_bytes && b.d_cap >= d_bytes) {
      x.h_buf = b.h;
      x.d_buf = b.d;
      x.h_cap = b.h_cap;
      x.d_cap = b.d_cap;
      c->pump_free.erase(c->pump_free.begin() + (long)k);
      return HICR_OK;
    }
  }
  auto pow2 = [](uint64_t v) {
    uint64_t p = 1 << 20;
    while (p < v) p <<= 1;
    return p;
  };
  const uint64_t hc = pow2(h_bytes), dc = pow2(d_bytes);
  if (hipHostMalloc(&x.h_buf, hc, hipHostMallocDefault) != hipSuccess) {
    x.h_buf = nullptr;
    return fail(c, HICR_ENOMEM, "pump staging (%llu bytes)", (unsigned long long)hc);
  }
  if (hipMalloc(&x.d_buf, dc) != hipSuccess) {
    (void)hipHostFree(x.h_buf);
    x.h_buf = x.d_buf = nullptr;
    return fail(c, HICR_ENOMEM, "pump tables (%llu bytes)", (unsigned long long)dc);
  }
  x.h_cap = hc;
  x.d_cap = dc;
  return HICR_OK;
}

// Return a pump's buffers for reuse (its launch has completed or never ran);
// at most 8 are kept, the smallest freed first.
static void give_pump_buf(hicr_ctx c, Extra &x) {
  if (!x.h_buf && !x.d_buf) return;
  c->pump_free.push_back(PumpBuf{x.h_buf, x.d_buf, x.h_cap, x.d_cap});
  x.h_buf = x.d_buf = nullptr;
  if (c->pump_free.size() > 8) {
    auto it = std::min_element(c->pump_free.begin(), c->pump_free.end(),
                               [](const PumpBuf &a, const PumpBuf &b) {
                                 return a.h_cap + a.d_cap < b.h_cap + b.d_cap;
                               });
    (void)hipFree(it->d);
    (void)hipHostFree(it->h);
    c->pump_free.erase(it);
  }
}

int pump_launch(hicr_ctx c, const std::vector<PumpStream> &st, const uint64_t *msg_off,
                const uint64_t *msg_size, uint64_t n_msgs, uint32_t *trace_dev, uint64_t *ts_dev,
                uint64_t timeout_ns, hipStream_t s, Extra *xout, bool dev_tables) {
  const uint32_t n = (uint32_t)st.size();
  if (n_msgs && (!msg_off || !msg_size)) return fail(c, HICR_EINVAL, "message arrays missing");
  // channels in order of first appearance
  std::vector<hicr_channel> chans;
  std::map<hicr_channel, uint32_t> chan_idx;
  std::map<std::pair<hicr_channel, uint32_t>, uint32_t> prod_stream;
  for (uint32_t i = 0; i < n; i++) {
    hicr_channel ch = st[i].channel;
    if (!ch || !registered(c, ch)) return fail(c, HICR_EINVAL, "stream %u: unknown channel", i);
    if (ch->cfg.endpoints != HICR_CH_DEVICE)
      return fail(c, HICR_EINVAL, "stream %u: channel has host endpoints", i);
    if (ch->broken) return fail(c, HICR_EINVAL, "stream %u: channel broken by an earlier error", i);
    if (ch->user_kernels)
      return fail(c, HICR_EINVAL, "stream %u: channel belongs to user kernels", i);
    if (st[i].producer >= ch->cfg.producers) return fail(c, HICR_EINVAL, "stream %u: producer", i);
    if (!prod_stream.emplace(std::make_pair(ch, st[i].producer), i).second)
      return fail(c, HICR_EINVAL, "stream %u: producer already has a stream", i);
    if (!chan_idx.count(ch)) {
      chan_idx[ch] = (uint32_t)chans.size();
      chans.push_back(ch);
    }
    if (st[i].first_msg > n_msgs || st[i].n_msgs > n_msgs - st[i].first_msg)
      return fail(c, HICR_ERANGE, "stream %u: messages outside the arrays", i);
    if (dev_tables) {
      // the producers check every message on the device
      if (ch->cfg.kind != HICR_CH_VAR)
        return fail(c, HICR_EINVAL, "stream %u: device message tables need a variable-size channel", i);
      continue;
    }
    uint64_t total = 0;
    for (uint64_t j = st[i].first_msg; j < st[i].first_msg + st[i].n_msgs; j++) {
      const uint64_t sz = msg_size[j], o = msg_off[j];
      if (ch->cfg.kind == HICR_CH_FIXED ? sz != ch->cfg.token_bytes : sz > ch->P)
        return fail(c, HICR_EINVAL, "stream %u message %llu: size %llu", i,
                    (unsigned long long)(j - st[i].first_msg), (unsigned long long)sz);
      if (o > st[i].src_size || sz > st[i].src_size - o)
        return fail(c, HICR_ERANGE, "stream %u message %llu outside its source", i,
                    (unsigned long long)(j - st[i].first_msg));
      total += sz;
    }
    if (total > st[i].out_size)
      return fail(c, HICR_ERANGE, "stream %u: output smaller than its %llu bytes", i,
                  (unsigned long long)total);
  }
  if (n == 0) return HICR_OK;
  // Consumer units.  A locking MPSC channel's shared ring is one unit (one
  // consumer, one total order).  Every other ring -- an SPSC channel's ring or
  // a non-locking MPSC producer's sub-ring -- has exactly one producer and is
  // consumed on its own; such rings are spread over as many consumer
  // workgroups as the device still holds, balanced by bytes (longest first),
  // so one channel's producers do not all wait on one workgroup.
  const uint32_t prod_wgs = (n + 3) / 4;
  const uint64_t cap = (uint64_t)c->n_cu * (uint64_t)c->pump_occ;
  // bytes per stream; with device tables the host balances by message count
  std::vector<uint64_t> stream_bytes(n, 0);
  for (uint32_t i = 0; i < n; i++) {
    if (dev_tables) {
      stream_bytes[i] = st[i].n_msgs;
      continue;
    }
    for (uint64_t j = st[i].first_msg; j < st[i].first_msg + st[i].n_msgs; j++)
      stream_bytes[i] += msg_size[j];
  }
  std::vector<uint64_t> chan_trace(chans.size());
  std::vector<uint64_t> stream_trace(n, 0);
  uint64_t trace_total = 0;
  for (uint32_t k = 0; k < chans.size(); k++) {
    chan_trace[k] = trace_total;
    for (uint32_t p = 0; p < chans[k]->cfg.producers; p++) {
      auto it = prod_stream.find(std::make_pair(chans[k], p));
      if (it == prod_stream.end()) continue;
      stream_trace[it->second] = trace_total;  // independent rings: producer after producer
      trace_total += st[it->second].n_msgs;
    }
  }
  std::vector<uint32_t> indep;  // streams whose ring is consumed on its own
  std::vector<uint64_t> chan_bytes(chans.size(), 0), chan_msgs(chans.size(), 0);
  std::vector<uint32_t> lock_chans;
  uint64_t all_bytes = 0;
  for (uint32_t k = 0; k < chans.size(); k++) {
    for (uint32_t p = 0; p < chans[k]->cfg.producers; p++) {
      auto it = prod_stream.find(std::make_pair(chans[k], p));
      if (it == prod_stream.end()) continue;
      chan_bytes[k] += stream_bytes[it->second];
      chan_msgs[k] += st[it->second].n_msgs;
      if (chans[k]->cfg.mode != HICR_CH_MPSC_LOCK) indep.push_back(it->second);
    }
    all_bytes += chan_bytes[k];
    if (chans[k]->cfg.mode == HICR_CH_MPSC_LOCK) lock_chans.push_back(k);
  }
  const uint64_t min_units = (indep.size() + kMaxProducers - 1) / kMaxProducers;
  if ((uint64_t)prod_wgs + lock_chans.size() + min_units > cap)
    return fail(c, HICR_EINVAL, "%llu workgroups do not fit the device at once (%d x %d)",
                (unsigned long long)(prod_wgs + lock_chans.size() + min_units), c->n_cu,
                c->pump_occ);
  // A locking MPSC ring is drained by a team sized to its share of the bytes
  // (every consumer workgroup should carry about the same), at most
  // kMaxTeam, and trimmed while the single-producer rings would not fit.
  const uint64_t budget = cap - prod_wgs;
  const uint64_t per_unit = std::max<uint64_t>(1, all_bytes / std::max<uint64_t>(1, budget));
  std::map<uint32_t, uint32_t> team;
  uint64_t team_total = 0;
  for (uint32_t k : lock_chans) {
    const uint64_t t = std::min<uint64_t>(kMaxTeam, std::max<uint64_t>(1, (chan_bytes[k] + per_unit - 1) / per_unit));
    team[k] = (uint32_t)t;
    team_total += t;
  }
  while (team_total + min_units > budget) {
    uint32_t big = lock_chans[0];
    for (uint32_t k : lock_chans)
      if (team[k] > team[big]) big = k;
    team[big]--;  // the fit check above guarantees one member per channel fits
    team_total--;
  }
  const uint32_t n_indep_units =
      (uint32_t)std::min<uint64_t>(indep.size(), budget - team_total);
  // longest first onto the least loaded unit (at most kMaxProducers rings each)
  std::vector<std::vector<uint32_t>> unit_streams(n_indep_units);
  {
    std::vector<uint32_t> order = indep;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return stream_bytes[x] > stream_bytes[y]; });
    using Load = std::pair<uint64_t, uint32_t>;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (uint32_t u = 0; u < n_indep_units; u++) heap.push(Load(0, u));
    for (uint32_t sid : order) {
      Load l = heap.top();
      heap.pop();
      unit_streams[l.second].push_back(sid);
      l.first += stream_bytes[sid] + 1;
      if (unit_streams[l.second].size() < kMaxProducers) heap.push(l);
    }
  }
  // tables
  std::vector<DevRing> rings;
  std::vector<DevChannel> dch;
  std::vector<uint32_t> sop;
  std::vector<DevStream> ds(n);
  std::vector<uint32_t> unit_of(n, 0), ring_of(n, 0);
  // device scratch of the locking teams: per channel a claim counter, a round
  // table (zeroed) and one 24-byte record per message
  std::vector<uint64_t> lock_claim_off, lock_side_off;
  uint64_t team_bytes = 0;
  for (uint32_t k : lock_chans) {
    lock_claim_off.push_back(team_bytes);
    team_bytes += 8 * (1 + chan_msgs[k] + team[k] + 1);
  }
  const uint64_t team_zero_bytes = team_bytes;
  for (uint32_t k : lock_chans) {
    lock_side_off.push_back(team_bytes);
    team_bytes += 24 * chan_msgs[k];
  }
  std::vector<uint32_t> lock_unit_first;  // first unit of each locking team
  for (uint32_t k = 0; k < chans.size(); k++) {
    hicr_channel ch = chans[k];
    if (ch->cfg.mode != HICR_CH_MPSC_LOCK) continue;
    DevChannel d{};
    d.mode = kModeMpscLock;
    d.n_rings = 1;
    d.first_ring = (uint32_t)rings.size();
    d.K = ch->cfg.producers;
    d.trace_base = chan_trace[k];
    d.prod_stream_base = (uint32_t)sop.size();
    DevRing rg = dev_ring(ch, 0);
    rg.base_m = ch->dev_msgs[0];
    rings.push_back(rg);
    uint32_t any = 0;
    for (uint32_t p = 0; p < d.K; p++) {
      auto it = prod_stream.find(std::make_pair(ch, p));
      if (it != prod_stream.end()) any = it->second;
    }
    for (uint32_t p = 0; p < d.K; p++) {
      auto it = prod_stream.find(std::make_pair(ch, p));
      sop.push_back(it != prod_stream.end() ? it->second : any);
      if (it != prod_stream.end()) {
        unit_of[it->second] = (uint32_t)dch.size();
        ring_of[it->second] = d.first_ring;
        d.total_msgs += st[it->second].n_msgs;
      }
    }
    lock_unit_first.push_back((uint32_t)dch.size());
    for (uint32_t m = 0; m < team[k]; m++) dch.push_back(d);  // claim/rounds set below
  }
  for (const auto &us : unit_streams) {
    DevChannel d{};
    d.mode = kModeSpsc;  // independent single-producer rings
    d.n_rings = (uint32_t)us.size();
    d.first_ring = (uint32_t)rings.size();
    d.K = d.n_rings;
    d.prod_stream_base = (uint32_t)sop.size();
    for (uint32_t sid : us) {
      hicr_channel ch = st[sid].channel;
      const uint32_t r = ch->cfg.mode == HICR_CH_MPSC_NOLOCK ? st[sid].producer : 0;
      unit_of[sid] = (uint32_t)dch.size();
      ring_of[sid] = (uint32_t)rings.size();
      rings.push_back(dev_ring(ch, r));
      sop.push_back(sid);
      d.total_msgs += st[sid].n_msgs;
    }
    dch.push_back(d);
  }
  const uint32_t nch = (uint32_t)dch.size();
  const uint32_t n_wgs = prod_wgs + nch;
  for (uint32_t i = 0; i < n; i++) {
    ds[i].channel = unit_of[i];
    ds[i].producer = st[i].producer;
    ds[i].ring = ring_of[i];
    ds[i].src_base = st[i].src_base;
    ds[i].out_base = st[i].out_base;
    ds[i].first_msg = st[i].first_msg;
    ds[i].n_msgs = st[i].n_msgs;
    ds[i].out_bytes = dev_tables ? st[i].out_size : stream_bytes[i];
    ds[i].trace_base = stream_trace[i];
    ds[i].src_bytes = st[i].src_size;
  }
  if (trace_dev) {
    int rc = check_dev_range(c, trace_dev, trace_total * 4, "trace_dev");
    if (rc != HICR_OK) return rc;
  }
  if (ts_dev) {
    int rc = check_dev_range(c, ts_dev, n_msgs * 16, "ts_dev");
    if (rc != HICR_OK) return rc;
  }
  std::vector<DevRole> roles;
  for (uint32_t i = 0; i < n; i += 4) {
    DevRole r{0, std::min<uint32_t>(4, n - i), {0, 0, 0, 0}};
    for (uint32_t w = 0; w < r.count; w++) r.ids[w] = i + w;
    roles.push_back(r);
  }
  for (uint32_t k = 0; k < nch; k++) roles.push_back(DevRole{1, 1, {k, 0, 0, 0}});
  // one upload: [err words | rings | channels | streams | sop | roles | msg_off | msg_size],
  // then the locking teams' device scratch (not uploaded; its head is zeroed)
  auto align = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
  uint64_t o_err = 0, o_ring = 256, o_ch = align(o_ring + rings.size() * sizeof(DevRing)),
           o_st = align(o_ch + dch.size() * sizeof(DevChannel)),
           o_sop = align(o_st + ds.size() * sizeof(DevStream)),
           o_role = align(o_sop + sop.size() * 4), o_off = align(o_role + roles.size() * sizeof(DevRole)),
           n_up = dev_tables ? 0 : n_msgs,  // message tables uploaded from the host
           o_size = align(o_off + n_up * 8), upload = align(o_size + n_up * 8),
           o_team = upload, total = align(o_team + team_bytes);
  Extra x;
  x.pump = true;
  int arc = take_pump_buf(c, upload, total, x);
  if (arc != HICR_OK) return arc;
  {
    // addresses of the locking teams' scratch, now that the buffer exists
    const uint64_t dbase = reinterpret_cast<uint64_t>(x.d_buf) + o_team;
    for (size_t t = 0; t < lock_chans.size(); t++) {
      const uint32_t u0 = lock_unit_first[t];
      rings[dch[u0].first_ring].side = dbase + lock_side_off[t];
      rings[dch[u0].first_ring].side_n = chan_msgs[lock_chans[t]];
      for (uint32_t m = 0; m < team[lock_chans[t]]; m++) {
        dch[u0 + m].claim = dbase + lock_claim_off[t];
        dch[u0 + m].rounds = dbase + lock_claim_off[t] + 8;
      }
    }
  }
  char *h = static_cast<char *>(x.h_buf);
  std::memset(h, 0, 256);
  // the host's abort request: a word of the pinned staging's zeroed head,
  // which nothing else writes while the pump runs; its address goes up with
  // the error words (err[4..5])
  const uint64_t abort_addr = reinterpret_cast<uint64_t>(h + kAbortHostOff);
  std::memcpy(h + o_err + 16, &abort_addr, 8);
  std::memcpy(h + o_ring, rings.data(), rings.size() * sizeof(DevRing));
  std::memcpy(h + o_ch, dch.data(), dch.size() * sizeof(DevChannel));
  std::memcpy(h + o_st, ds.data(), ds.size() * sizeof(DevStream));
  std::memcpy(h + o_sop, sop.data(), sop.size() * 4);
  std::memcpy(h + o_role, roles.data(), roles.size() * sizeof(DevRole));
  if (n_up) {
    std::memcpy(h + o_off, msg_off, n_up * 8);
    std::memcpy(h + o_size, msg_size, n_up * 8);
  }
  char *d = static_cast<char *>(x.d_buf);
  PumpArgs a;
  a.rings = reinterpret_cast<const DevRing *>(d + o_ring);
  a.chans = reinterpret_cast<const DevChannel *>(d + o_ch);
  a.streams = reinterpret_cast<const DevStream *>(d + o_st);
  a.stream_of_prod = reinterpret_cast<const uint32_t *>(d + o_sop);
  a.roles = reinterpret_cast<const DevRole *>(d + o_role);
  a.msg_off = dev_tables ? msg_off : reinterpret_cast<const uint64_t *>(d + o_off);
  a.msg_size = dev_tables ? msg_size : reinterpret_cast<const uint64_t *>(d + o_size);
  a.trace = trace_dev;
  a.ts_push = ts_dev;
  a.ts_pop = ts_dev ? ts_dev + n_msgs : nullptr;
  a.err = reinterpret_cast<uint32_t *>(d + o_err);
  const uint64_t tns = timeout_ns ? timeout_ns : 10'000'000'000ull;
  a.timeout_ticks = tns / 10;  // 100 MHz device clock
  // Earlier pumps still in flight on other streams: this one follows every
  // one that drives one of its rings, and the oldest others until all
  // pumps that can be in flight together fit the device at once.
  hipError_t e = hipSuccess;
  {
    std::vector<LiveLaunch> live;
    for (const PumpLive &p : c->pump_live) {
      LiveLaunch l;
      l.wgs = p.wgs;
      l.done = hipEventQuery(p.ev) == hipSuccess;
      l.same_stream = p.stream == s;
      l.shares_channel = false;
      for (hicr_channel ch : p.chans)
        if (chan_idx.count(ch)) l.shares_channel = true;
      live.push_back(l);
    }
    for (size_t i : residency_waits(live, n_wgs, cap))
      if (e == hipSuccess) e = hipStreamWaitEvent(s, c->pump_live[i].ev, 0);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(d, h, upload, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && team_zero_bytes) e = hipMemsetAsync(d + o_team, 0, team_zero_bytes, s);
  if (e == hipSuccess) e = launch_pump(a, n_wgs, s);
  // error words come back into the (no longer needed) head of the staging
  if (e == hipSuccess) e = hipMemcpyAsync(h, d, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&x.ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(x.ev, s);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s);
    if (x.ev) (void)hipEventDestroy(x.ev);
    give_pump_buf(c, x);
    return hip_fail(c, e, "launching the channel pump");
  }
  x.abort_word = reinterpret_cast<uint32_t *>(h + kAbortHostOff);
  x.chans = chans;
  {
    PumpLive pl;
    pl.ev = x.ev;
    pl.stream = s;
    pl.wgs = n_wgs;
    pl.chans = chans;
    c->pump_live.push_back(pl);
  }
  // the rings' message counters when the next pump starts
  for (uint32_t i = 0; i < n; i++) {
    hicr_channel ch = st[i].channel;
    const uint32_t r = ch->cfg.mode == HICR_CH_MPSC_NOLOCK ? st[i].producer : 0;
    ch->dev_msgs[r] += st[i].n_msgs;
  }
  {
    std::lock_guard<std::mutex> ga(c->abort_mu);
    c->abort_words.push_back(x.abort_word);
  }
  *xout = x;
  return HICR_OK;
}

// Outcome of a finished pump (its event has completed): release its buffers
// and report a device-side error.
int pump_finish(hicr_ctx c, Extra &x) {
  int rc = HICR_OK;
  for (size_t i = 0; i < c->pump_live.size(); i++)
    if (c->pump_live[i].ev == x.ev) {
      c->pump_live.erase(c->pump_live.begin() + i);
      break;
    }
  const uint32_t *err = static_cast<const uint32_t *>(x.h_buf);
  if (err[0] & kErrCorrupt) rc = fail(c, HICR_EDEVICE, "a channel pump read a malformed entry");
  else if (err[0] & kErrTimeout) rc = fail(c, HICR_ETIMEDOUT, "a channel pump made no progress");
  else if (err[1]) rc = fail(c, HICR_EDEVICE, "a channel pump was aborted");
  if (err[0] || err[1])
    for (hicr_channel ch : x.chans) ch->broken = true;
  {
    std::lock_guard<std::mutex> g(c->abort_mu);
    c->abort_words.erase(std::remove(c->abort_words.begin(), c->abort_words.end(), x.abort_word),
                         c->abort_words.end());
  }
  (void)hipEventDestroy(x.ev);
  give_pump_buf(c, x);
  x = Extra();
  return rc;
}

void destroy_pump_bufs(hicr_ctx c) {
  for (PumpBuf &b : c->pump_free) {
    if (b.d) (void)hipFree(b.d);
    if (b.h) (void)hipHostFree(b.h);
  }
  c->pump_free.clear();
}

uint64_t channel_payload_limit(hicr_channel ch) {
  return ch->cfg.kind == HICR_CH_FIXED ? ch->cfg.token_bytes : ch->P;
}

}  // namespace hicr

extern "C" {

int hicr_channel_pump(hicr_ctx c, const hicr_stream *st, uint32_t n, const hicr_pump_io *io,
                      void *stream) {
  return guarded([&]() -> int {
    if (!c || !io || (n && !st) || (io->flags & ~HICR_PUMP_DEVICE_TABLES) || io->reserved)
      return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    std::vector<PumpStream> ps(n);
    for (uint32_t i = 0; i < n; i++) {
      int rc = check_hbm_slot(c, st[i].src, 1, "stream source");
      if (rc != HICR_OK) return rc;
      rc = check_hbm_slot(c, st[i].out, 1, "stream output");
      if (rc != HICR_OK) return rc;
      ps[i].channel = st[i].channel;
      ps[i].producer = st[i].producer;
      ps[i].src_base = c->slots[st[i].src].base;
      ps[i].src_size = c->slots[st[i].src].size;
      ps[i].out_base = c->slots[st[i].out].base;
      ps[i].out_size = c->slots[st[i].out].size;
      ps[i].first_msg = st[i].first_msg;
      ps[i].n_msgs = st[i].n_msgs;
    }
    Extra x;
    int rc = pump_launch(c, ps, io->msg_src_off, io->msg_size, io->n_msgs, io->trace_dev,
                         io->ts_dev, io->timeout_ns,
                         stream ? static_cast<hipStream_t>(stream) : c->stream, &x,
                         (io->flags & HICR_PUMP_DEVICE_TABLES) != 0);
    if (rc == HICR_OK && x.ev) c->extra.push_back(x);
    return rc;
  });
}

int hicr_channel_device_view(hicr_channel ch, uint32_t ring, hicr_dev_ring *out) {
  return guarded([&]() -> int {
    if (!ch || !out) return HICR_EINVAL;
    hicr_ctx c = ch->ctx;
    std::lock_guard<std::mutex> g(c->mu);
    if (!registered(c, ch)) return HICR_EINVAL;
    if (ch->cfg.endpoints != HICR_CH_DEVICE) return fail(c, HICR_EINVAL, "host-endpoint channel");
    if (ch->cfg.mode == HICR_CH_MPSC_LOCK)
      return fail(c, HICR_EUNSUPPORTED, "locking MPSC rings are driven by the pump only");
    if (ring >= ch->n_rings) return fail(c, HICR_EINVAL, "no ring %u", ring);
    if (ch->broken) return fail(c, HICR_EINVAL, "channel broken by an earlier error");
    const DevRing r = dev_ring(ch, ring);
    out->payload = r.payload;
    out->P = r.P;
    out->entries = r.entries;
    out->E = r.E;
    out->coord = r.coord;
    out->producer = ch->cfg.mode == HICR_CH_MPSC_NOLOCK ? ring : 0;
    out->pad = 0;
    ch->user_kernels = true;
    return HICR_OK;
  });
}

int hicr_channel_abort(hicr_ctx c) {
  return guarded([&]() -> int {
    if (!c) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->abort_mu);  // not c->mu: a fence may hold it
    // a store into each running pump's pinned abort word: no queue is
    // involved, so the request cannot wait behind the pump it is meant to
    // stop (streams share the device's few hardware queues)
    for (uint32_t *w : c->abort_words) __atomic_store_n(w, 1u, __ATOMIC_RELEASE);
    return HICR_OK;
  });
}

}  // extern "C"
