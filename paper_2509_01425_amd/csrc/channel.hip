// channel.hip -- gfx950 kernels of the ring channels (HiCR Sec. 4.3).
//
// Protocol (per ring; counters monotone, see chan.h):
//   producer: wait until the consumer's released counters leave room for the
//             message (entries tm - hm < E, bytes tb - hb + s <= P), write the
//             payload at byte position tb mod P (split across the ring end),
//             write the entry, release fence, publish tm + 1;
//   consumer: acquire-read tm; while tm > hm read entry hm mod E and the
//             payload at hb mod P, then release fence and publish hb + s and
//             hm + 1 -- the notification that frees the producer's room.
// Locking MPSC: a ticket lock (FIFO-fair) guards the room check and the
// reservation of [rb, rb + s) / entry rm; the copy runs outside the lock and
// publication follows ticket order, so the shared ring holds one total order
// and never overflows.  Non-locking MPSC: one ring per producer; the
// consumer polls them round robin.
//
// pump_kernel is persistent: every workgroup is either four independent
// producer waves (one stream each) or one consumer (all four waves).  Waits
// poll with relaxed device-scope loads and take one acquire fence once the
// condition holds (an acquire per poll would invalidate the L2 on every
// spin).  Producers copy up to 16 messages at a time (8 on a locking ring),
// message by message; the producer of a long stream through a ring of its
// own holds full batches of 16 unpublished, up to a ring's worth of entries
// (E / 16 batches), and publishes them with one release (fewer releases, each
// of which writes back the XCD's L2); consumers take up to 32 per release
// across all of their rings and copy each batch as one index space of
// 16-byte vectors.  Producers check every message against their stream's
// slots before moving a byte.  The host launches no more workgroups than the
// device holds at once, and every wait gives up after a no-progress time-out
// or on the abort word, so every wave exits.
#include "chan.h"

namespace hicr {

#define GLOBAL __attribute__((address_space(1)))
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef v4u v4u_any __attribute__((aligned(1)));


__device__ __forceinline__ uint64_t ld_acq(uint64_t a) {
  return __hip_atomic_load((uint64_t *)a, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_rlx(uint64_t a) {
  return __hip_atomic_load((uint64_t *)a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(uint64_t a, uint64_t v) {
  __hip_atomic_store((uint64_t *)a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t a, uint64_t v) {
  __hip_atomic_store((uint64_t *)a, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// A 16-byte payload store (ring or output).
__device__ __forceinline__ void st16(uint64_t a, v4u v) { *(GLOBAL v4u *)a = v; }

// Copy n bytes d <- s with a team of TEAM threads (t = rank in the team):
// destination-aligned 16-byte stores, source at any alignment, the at most
// 15 head and 15 tail bytes one by one.  TEAM >= 64.  The code has no
// per-lane branch: a lane past the last vector copies the last vector again,
// and every lane copies one byte (lanes 0-15 the head bytes, 16-31 the tail
// bytes, a repeated byte once a range is used up, the request's first byte
// on the other lanes), so repeated stores write equal values and nothing
// outside the request is touched.  Without lane branches the compiler issues
// a round's U loads back to back and never waits for an earlier store; a
// bounds test on every access made it wait for each access in turn (about
// three memory latencies per round instead of one).
template <int TEAM, int U>
__device__ __forceinline__ void team_copy(uint64_t d, uint64_t s, uint64_t n, uint32_t t) {
  if (n == 0) return;
  uint64_t a0 = (d + 15) & ~(uint64_t)15;
  if (a0 > d + n) a0 = d + n;
  uint64_t a1 = (d + n) & ~(uint64_t)15;
  if (a1 < a0) a1 = a0;
  const uint64_t nh = a0 - d, nt = d + n - a1;
  uint64_t bo = 0;  // this lane's byte, as an offset into the request
  if (t < 16)
    bo = nh ? (t < nh ? t : nh - 1) : 0;
  else if (t < 32)
    bo = nt ? (a1 - d) + (t - 16 < nt ? t - 16 : nt - 1) : 0;
  const unsigned char byte = *(const GLOBAL unsigned char *)(s + bo);
  const uint64_t nv = (a1 - a0) >> 4;
  const uint64_t s16 = s + nh;
  constexpr uint64_t step = (uint64_t)TEAM * U;
  for (uint64_t b = 0; b < nv; b += step) {
    v4u r[U];
    uint64_t o[U];
#pragma unroll
    for (int k = 0; k < U; k++) {
      const uint64_t i = b + t + (uint64_t)k * TEAM;
      o[k] = 16 * (i < nv ? i : nv - 1);
    }
#pragma unroll
    for (int k = 0; k < U; k++) r[k] = *(const GLOBAL v4u_any *)(s16 + o[k]);
#pragma unroll
    for (int k = 0; k < U; k++) st16(a0 + o[k], r[k]);
  }
  *(GLOBAL unsigned char *)(d + bo) = byte;
}

// Payload write / read at ring position pos, split across the ring end.
template <int TEAM, int U>
__device__ __forceinline__ void ring_put(const DevRing &r, uint64_t pos, uint64_t src, uint64_t n,
                                         uint32_t t) {
  uint64_t first = r.P - pos < n ? r.P - pos : n;
  team_copy<TEAM, U>(r.payload + pos, src, first, t);
  if (n > first) team_copy<TEAM, U>(r.payload, src + first, n - first, t);
}

// No-progress watchdog for spin waits.
// The error and abort words are shared by every wave of the pump, so a wave
// looks at them at most once per kWatchTicks of its own waiting (10 us of the
// 100 MHz clock) instead of on every poll: thousands of spinning waves
// reading one address would otherwise queue at one memory channel.  The
// host asks for an abort in pinned host memory (a plain store, so that no
// queue has to run beside the pump; err[4..5] hold that word's address): a
// wave reads it over the host link only in one of every 1,024 windows of
// 1,024 ticks (about once per 10 ms of its own waiting), the windows
// staggered over the waves so that their reads do not arrive together and
// a pump with many waiting waves sees the request within tens of
// microseconds, and passes a request on to err[1], which every wave reads.
// (Measured on the channel workload: reading it in one window of 128, all
// waves in the same one, cost 3 % of the pump's rate; one of 1,024, 0.3-1 %.)
constexpr uint64_t kWatchTicks = 1000;

struct Watch {
  uint64_t deadline, span;
  uint32_t *err;
  uint64_t next;
  __device__ void progress() { deadline = wall_clock64() + span; }
  // true when the wait must stop (time-out recorded, or abort requested)
  __device__ bool expired() {
    const uint64_t now = wall_clock64();
    if (now < next) return false;
    next = now + kWatchTicks;
    const uint32_t salt = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if ((((now >> 10) + salt) & 1023) == 0) {
      const uint32_t *host = reinterpret_cast<const uint32_t *>(__hip_atomic_load(
          reinterpret_cast<uint64_t *>(err + 4), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (host && __hip_atomic_load(host, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
        if (__lane_id() == 0)
          __hip_atomic_store(&err[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
      }
    }
    if (__hip_atomic_load(&err[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
        __hip_atomic_load(&err[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return true;
    if (now > deadline) {
      __hip_atomic_fetch_or(&err[0], kErrTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return true;
    }
    return false;
  }
};

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  return ((uint64_t)__shfl((unsigned)(v >> 32), src) << 32) | (uint64_t)__shfl((unsigned)v, src);
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_scan(uint64_t v, uint32_t lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t t = ((uint64_t)__shfl_up((unsigned)(v >> 32), o) << 32) | __shfl_up((unsigned)v, o);
    if (lane >= (uint32_t)o) v += t;
  }
  return v;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A contiguous piece of a batched copy: n bytes d <- s.  a0 is the first
// 16-byte-aligned destination byte inside it (clipped), nv its 16-byte body
// vectors, v0 the body vectors of all earlier segments.
struct Seg {
  uint64_t d, s, n, a0, nv, v0;
};

__device__ __forceinline__ Seg make_seg(uint64_t d, uint64_t s, uint64_t n) {
  Seg g;
  g.d = d;
  g.s = s;
  g.n = n;
  uint64_t a0 = (d + 15) & ~(uint64_t)15;
  if (a0 > d + n) a0 = d + n;
  uint64_t a1 = (d + n) & ~(uint64_t)15;
  if (a1 < a0) a1 = a0;
  g.a0 = a0;
  g.nv = (a1 - a0) >> 4;
  g.v0 = 0;
  return g;
}

// All TEAM threads copy nseg segments (held in LDS, every one non-empty, at
// most kMaxSegs) as one index space of 16-byte vectors, so a batch of small
// messages costs about one memory round trip instead of one per message.
// Branch-free like team_copy: the head and tail bytes (slot 32 g + j: j < 16
// head byte j of segment g, else tail byte j - 16) and the vectors are
// clamped into range, so repeated copies write equal values, and a vector's
// segment is found by a fixed binary search (log2 kMaxSegs steps) over the segments'
// first vectors (v0) instead of a data-dependent loop; the compiler then
// issues a round's U loads back to back.
constexpr uint32_t kMaxSegs = 64;  // a power of two
template <int TEAM, int U>
__device__ void seg_copy(const Seg *sg, uint32_t nseg, uint64_t total_v, uint32_t t) {
  if (nseg == 0) return;
  constexpr int kB = (32 * kMaxSegs + TEAM - 1) / TEAM;  // byte slots per thread
  unsigned char bv[kB];
  uint64_t bd[kB];
#pragma unroll
  for (int q = 0; q < kB; q++) {
    uint32_t x = t + (uint32_t)q * TEAM;
    if (x > nseg * 32 - 1) x = nseg * 32 - 1;
    const Seg &g = sg[x >> 5];
    const uint32_t j = x & 31;
    const uint64_t nh = g.a0 - g.d, a1 = g.a0 + 16 * g.nv, nt = g.d + g.n - a1;
    uint64_t off;
    if (j < 16)
      off = nh ? (j < nh ? j : nh - 1) : 0;
    else
      off = nt ? (a1 - g.d) + (j - 16 < nt ? j - 16 : nt - 1) : 0;
    bv[q] = *(const GLOBAL unsigned char *)(g.s + off);
    bd[q] = g.d + off;
  }
#pragma unroll
  for (int q = 0; q < kB; q++) *(GLOBAL unsigned char *)(bd[q]) = bv[q];
  for (uint64_t b = 0; b < total_v; b += (uint64_t)TEAM * U) {
    uint64_t sa[U], da[U];
#pragma unroll
    for (int k = 0; k < U; k++) {
      uint64_t v = b + t + (uint64_t)k * TEAM;
      if (v > total_v - 1) v = total_v - 1;
      uint32_t c = 0;  // last segment with v0 <= v
#pragma unroll
      for (uint32_t st = kMaxSegs / 2; st; st >>= 1) {
        const uint32_t i = c + st < nseg ? c + st : nseg - 1;
        c = (c + st < nseg && sg[i].v0 <= v) ? c + st : c;
      }
      const Seg &g = sg[c];
      const uint64_t w = 16 * (v - g.v0);
      sa[k] = g.s + (g.a0 - g.d) + w;
      da[k] = g.a0 + w;
    }
    v4u r[U];
#pragma unroll
    for (int k = 0; k < U; k++) r[k] = *(const GLOBAL v4u_any *)(sa[k]);
#pragma unroll
    for (int k = 0; k < U; k++) st16(da[k], r[k]);
  }
}

// Messages a producer publishes at once: 16 on a ring of its own, 8 on a
// locking MPSC ring, where a larger reservation keeps the other producers
// waiting for room longer (measured: 16 gave +15% on the non-locking pump and
// -5% on the locking one).
constexpr uint32_t kProdBatch = 16;
constexpr uint32_t kProdBatchLocking = 8;
constexpr uint32_t kConsBatch = 32;  // messages a consumer takes at once
static_assert(2 * kConsBatch <= kMaxSegs, "a consumer batch is at most 2 segments per message");

// One producer wave drives one stream: it takes as many of its next messages
// as the ring has room for (up to kProdBatch, or kProdBatchLocking), copies
// them as one batch and writes their entries.  A locking ring publishes every
// batch (in reservation order).  On a ring of its own, a stream of more than
// four rings' worth of entries keeps full batches unpublished, up to
// E / kProdBatch of them, and publishes them with one release; when the next
// message does not fit, it publishes what it holds before it waits (the
// consumer cannot free room for messages it has not seen).  Measured on the
// channel configuration (~650 messages per stream), one process alternating:
// 3,564-3,680 GB/s holding up to four batches against 2,873-3,207 with a
// release per batch, message latency p99 0.9 ms against 2.2-2.6 ms.  Short
// streams publish every batch: holding in the serving loop's bursts (at most
// 256 messages) raised its latency p99 from 1.9 to 3.1 ms, and holding only
// while the consumer had a batch left to work on still to 2.3 ms, as a burst
// loses the overlap of its producer and consumer.
__device__ void run_producer(const PumpArgs &a, uint32_t sid_in, uint32_t lane, Seg *sg) {
  // the stream id is the same in every lane of the wave; saying so lets the
  // stream and ring descriptors live in scalar registers
  const uint32_t sid = __builtin_amdgcn_readfirstlane(sid_in);
  const DevStream st = a.streams[sid];
  const DevRing r = a.rings[st.ring];
  const bool locking = a.chans[st.channel].mode == kModeMpscLock;
  const uint64_t c = r.coord;
  const uint64_t tm_a = c + offsetof(RingCoord, prod), hm_a = c + offsetof(RingCoord, cons),
                 hb_a = hm_a + 8, tk_a = c + offsetof(RingCoord, lock), sv_a = tk_a + 8,
                 rm_a = tk_a + 16, rb_a = tk_a + 24;
  // rings are empty when a pump starts: the producer side resumes at the
  // consumer's released counters
  uint64_t tm = ld_acq(tm_a), tb = ld_acq(hb_a);
  Watch w{0, a.timeout_ticks, a.err, 0};
  w.progress();
  uint64_t m = 0;
  uint64_t out_run = 0;  // output bytes of this stream's earlier messages
  const uint64_t max_held =
      locking || st.n_msgs <= 4 * r.E ? 1 : (r.E / kProdBatch > 1 ? r.E / kProdBatch : 1);
  uint64_t pub_m = 0;  // messages published
  uint64_t held = 0;   // full batches copied and not yet published
  // the release covers the payload and entries of every message since the
  // last publication; then the counters move past them
  auto publish = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (a.ts_push)
      for (uint64_t k = lane; k < m - pub_m; k += 64) a.ts_push[st.first_msg + pub_m + k] = wall_clock64();
    if (lane == 0) {
      // a ring of its own also publishes its byte counter, the form user
      // kernels (hicr_device.h) resume from
      st_rlx(tm_a + 8, tb);
      st_rlx(tm_a, tm);
    }
    pub_m = m;
    held = 0;
  };
  while (m < st.n_msgs) {
    // sizes and offsets of the next messages of this batch, one per lane
    const bool have = lane < (locking ? kProdBatchLocking : kProdBatch) && m + lane < st.n_msgs;
    const uint64_t sz = have ? a.msg_size[st.first_msg + m + lane] : 0;
    const uint64_t off = have ? a.msg_off[st.first_msg + m + lane] : 0;
    const uint64_t incl = wave_scan(sz, lane);
    // every message is checked before a byte of it moves (the host has not
    // seen message tables that live on the device): it fits the ring, its
    // source range lies in the stream's source slot, its output in the
    // output slot
    const bool bad = have && (sz > r.P || off > st.src_bytes || sz > st.src_bytes - off ||
                              out_run + incl > st.out_bytes);
    if (__ballot(bad)) {
      if (lane == 0)
        __hip_atomic_fetch_or(&a.err[0], kErrCorrupt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    uint64_t ticket = 0;
    if (locking) {
      if (lane == 0)
        ticket = __hip_atomic_fetch_add((uint64_t *)tk_a, 1ull, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
      ticket = shfl64(ticket, 0);
      while (ld_rlx(sv_a) != ticket) {
        __builtin_amdgcn_s_sleep(1);
        if (w.expired()) return;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    uint64_t my_tm = locking ? ld_rlx(rm_a) : tm;
    uint64_t my_tb = locking ? ld_rlx(rb_a) : tb;
    // wait until at least the first message fits, then take every leading
    // message that fits in the room seen
    uint64_t hm, hb;
    const uint64_t s0 = shfl64(sz, 0);
    for (;;) {
      hm = shfl64(ld_rlx(hm_a), 0);  // one view of the consumer for the whole wave
      hb = shfl64(ld_rlx(hb_a), 0);
      if (my_tm - hm < r.E && my_tb - hb + s0 <= r.P) break;
      if (held) publish();
      __builtin_amdgcn_s_sleep(2);
      if (w.expired()) return;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the consumer's reads are done
    const bool fits = have && (my_tm + lane + 1 - hm <= r.E) && (my_tb + incl - hb <= r.P);
    const uint64_t fm = __ballot(fits);
    const uint32_t j = (uint32_t)__ffsll((unsigned long long)~fm) - 1;  // leading fitting lanes
    const uint64_t bytes = shfl64(incl, (int)j - 1);
    if (locking && lane == 0) {
      st_rlx(rm_a, my_tm + j);
      st_rlx(rb_a, my_tb + bytes);
      st_rel(sv_a, ticket + 1);
    }
    // entries (and, on a locking ring, the records the consumer team reads)
    // are written now, before the copy, so sizes and offsets need not stay
    // in registers across it; the release before publication covers them
    if (lane < j) {
      *(GLOBAL uint64_t *)(r.entries + 8 * ((my_tm + lane) % r.E)) =
          sz | ((uint64_t)st.producer << 48);
      if (locking) {
        // the message's record for the consumer team: ring byte position,
        // output address, message index (a counter outside this pump's
        // records means the ring's state is not what the host planned for)
        const uint64_t idx = my_tm + lane - r.base_m;
        if (idx < r.side_n) {
          uint64_t *rec = (uint64_t *)(r.side + 24 * idx);
          rec[0] = my_tb + incl - sz;
          rec[1] = st.out_base + out_run + incl - sz;
          rec[2] = st.first_msg + m + lane;
        } else {
          __hip_atomic_fetch_or(&a.err[0], kErrCorrupt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    // segments: message l of the batch -> ring bytes at (my_tb + excl_l) mod P
    if (lane < j) {
      const uint64_t pos = (my_tb + incl - sz) % r.P;
      const uint64_t first = r.P - pos < sz ? r.P - pos : sz;
      sg[2 * lane] = make_seg(r.payload + pos, st.src_base + off, first);
      sg[2 * lane + 1] = make_seg(r.payload, st.src_base + off + first, sz - first);
    }
    wave_sync();
    // one segment after another, each in full rounds of 4 KiB (a batch as
    // one index space of vectors needs a search per vector, which kept the
    // loads of a round from overlapping)
    for (uint32_t g = 0; g < 2 * j; g++) team_copy<64, 4>(sg[g].d, sg[g].s, sg[g].n, lane);
    if (locking) {
      // publish in reservation order, carrying the predecessors' writes
      while (ld_rlx(tm_a) != my_tm) {
        __builtin_amdgcn_s_sleep(1);
        if (w.expired()) return;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      if (a.ts_push && lane < j) a.ts_push[st.first_msg + m + lane] = wall_clock64();
      if (lane == 0) st_rlx(tm_a, my_tm + j);
    }
    tm = my_tm + j;
    tb = my_tb + bytes;
    m += j;
    out_run += bytes;
    if (!locking) {
      if (held + 1 < max_held && j == kProdBatch && m < st.n_msgs)
        held++;
      else
        publish();
    }
    wave_sync();
    w.progress();
  }
}

// One consumer workgroup drains a set of independent rings, each with a
// single producer stream (SPSC rings, non-locking MPSC sub-rings): each round
// it looks at all of its rings at once, takes up to kConsBatch published
// messages (round robin over rings), copies them as one batch to their
// streams' outputs and releases each ring's room with one store pair.
__device__ void run_consumer(const PumpArgs &a, uint32_t cid, uint32_t tid) {
  __shared__ uint64_t s_hm[kMaxProducers], s_hb[kMaxProducers];
  __shared__ uint64_t s_outpos[kMaxProducers], s_cnt[kMaxProducers];
  __shared__ uint32_t s_take[kMaxProducers];
  __shared__ uint64_t s_ent[kConsBatch];
  __shared__ uint32_t s_ring_of[kConsBatch];
  __shared__ uint64_t s_idx_of[kConsBatch];
  __shared__ uint64_t s_rbytes[kMaxProducers];
  __shared__ Seg s_seg[2 * kConsBatch];
  __shared__ uint32_t s_k, s_stop, s_nseg;
  __shared__ uint64_t s_total_v;
  // per-ring and per-producer tables, staged once so the planning loop
  // below touches LDS only
  __shared__ uint64_t s_rpay[kMaxProducers], s_rent[kMaxProducers], s_rcoord[kMaxProducers];
  __shared__ uint64_t s_pout[kMaxProducers], s_pbytes[kMaxProducers];
  __shared__ uint64_t s_pfirst[kMaxProducers], s_pn[kMaxProducers], s_ptrace[kMaxProducers];
  __shared__ uint64_t s_rP[kMaxProducers], s_rE[kMaxProducers];
  __shared__ uint32_t s_psid[kMaxProducers];
  const DevChannel ch = a.chans[cid];
  const uint32_t lane = tid & 63, wave = tid >> 6;
  for (uint32_t i = tid; i < ch.n_rings; i += kPumpBlock) {
    const DevRing rg = a.rings[ch.first_ring + i];
    const uint64_t c = rg.coord + offsetof(RingCoord, cons);
    s_hm[i] = ld_acq(c);
    s_hb[i] = ld_acq(c + 8);
    s_rpay[i] = rg.payload;
    s_rent[i] = rg.entries;
    s_rcoord[i] = rg.coord;
    s_rP[i] = rg.P;
    s_rE[i] = rg.E;
  }
  for (uint32_t p = tid; p < ch.K; p += kPumpBlock) {
    const uint32_t sid = a.stream_of_prod[ch.prod_stream_base + p];
    const DevStream so = a.streams[sid];
    s_psid[p] = sid;
    s_pout[p] = so.out_base;
    s_pbytes[p] = so.out_bytes;
    s_pfirst[p] = so.first_msg;
    s_pn[p] = so.n_msgs;
    s_ptrace[p] = so.trace_base;
    s_outpos[p] = 0;
    s_cnt[p] = 0;
  }
  __syncthreads();
  Watch w{0, a.timeout_ticks, a.err, 0};
  w.progress();
  uint64_t done = 0;
  uint32_t rr = 0;
  while (done < ch.total_msgs) {
    if (wave == 0) {
      uint64_t av = 0;
      uint32_t ri = 0;
      bool stop = false;
      for (;;) {
        av = 0;
        if (lane < ch.n_rings) {
          ri = (rr + lane) % ch.n_rings;
          av = ld_rlx(s_rcoord[ri] + offsetof(RingCoord, prod)) - s_hm[ri];
        }
        if (__ballot(av > 0)) break;
        __builtin_amdgcn_s_sleep(2);
        if (w.expired()) {
          stop = true;
          break;
        }
      }
      // quotas in ring order starting at rr: take while the batch has room
      const uint64_t left = ch.total_msgs - done;
      const uint64_t cap = left < kConsBatch ? left : kConsBatch;
      const uint64_t want = av < cap ? av : cap;
      const uint64_t incl = wave_scan(want, lane);
      uint64_t take = 0;
      if (incl - want < cap) take = (incl <= cap) ? want : cap - (incl - want);
      if (lane < ch.n_rings) s_take[ri] = (uint32_t)take;
      const uint64_t k = shfl64(wave_scan(take, lane), 63);
      if (lane == 0) {
        s_stop = stop;
        s_k = (uint32_t)k;
      }
    }
    __syncthreads();
    if (s_stop) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const uint32_t k = s_k;
    // message i of the batch: ring and index within it (rings in order from rr)
    if (tid == 0) {
      uint32_t i = 0;
      for (uint32_t q = 0; q < ch.n_rings && i < k; q++) {
        const uint32_t ri = (rr + q) % ch.n_rings;
        for (uint32_t x = 0; x < s_take[ri]; x++, i++) {
          s_ring_of[i] = ri;
          s_idx_of[i] = s_hm[ri] + x;
        }
      }
    }
    __syncthreads();
    if (tid < k) {
      const uint32_t ri = s_ring_of[tid];
      s_ent[tid] = *(const GLOBAL uint64_t *)(s_rent[ri] + 8 * (s_idx_of[tid] % s_rE[ri]));
    }
    __syncthreads();
    if (tid == 0) {
      // plan the copies; entries are checked against the plan first, so a
      // malformed entry stops the pump instead of writing out of bounds
      uint32_t bad = 0, nseg = 0;
      for (uint32_t q = 0; q < ch.n_rings; q++) s_rbytes[q] = 0;
      for (uint32_t i = 0; i < k; i++) {
        const uint32_t ri = s_ring_of[i];
        const uint64_t e = s_ent[i];
        const uint64_t sz = e & kEntrySizeMask;
        const uint32_t p = ri;  // ring q carries producer stream q of the unit
        const uint64_t P = s_rP[ri];
        if (sz > P || s_outpos[p] + sz > s_pbytes[p] || s_cnt[p] >= s_pn[p]) {
          bad = 1;
          break;
        }
        const uint64_t pos = (s_hb[ri] + s_rbytes[ri]) % P;
        const uint64_t first = P - pos < sz ? P - pos : sz;
        const uint64_t dst = s_pout[p] + s_outpos[p];
        if (first) s_seg[nseg++] = make_seg(dst, s_rpay[ri] + pos, first);
        if (sz > first) s_seg[nseg++] = make_seg(dst + first, s_rpay[ri], sz - first);
        s_rbytes[ri] += sz;
        s_outpos[p] += sz;
        if (a.trace) a.trace[s_ptrace[p] + s_cnt[p]] = s_psid[p];
        if (a.ts_pop) a.ts_pop[s_pfirst[p] + s_cnt[p]] = wall_clock64();
        s_cnt[p] += 1;
      }
      uint64_t v = 0;
      for (uint32_t g = 0; g < nseg; g++) {
        s_seg[g].v0 = v;
        v += s_seg[g].nv;
      }
      s_nseg = nseg;
      s_total_v = v;
      if (bad) {
        __hip_atomic_fetch_or(&a.err[0], kErrCorrupt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_stop = 1;
      }
    }
    __syncthreads();
    if (s_stop) break;
    seg_copy<kPumpBlock, 4>(s_seg, s_nseg, s_total_v, tid);
    __syncthreads();  // every read of the rings has completed
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      for (uint32_t q = 0; q < ch.n_rings; q++) {
        const uint32_t t = s_take[q];
        if (!t) continue;
        const uint64_t c = s_rcoord[q] + offsetof(RingCoord, cons);
        s_hb[q] += s_rbytes[q];
        s_hm[q] += t;
        st_rlx(c + 8, s_hb[q]);
        st_rlx(c, s_hm[q]);
      }
    }
    done += k;
    rr = (rr + 1) % ch.n_rings;
    w.progress();
  }
  __threadfence();
}

// A locking MPSC ring consumed by a team of workgroups.  The ring holds one
// total order; it is cut into rounds of consecutive messages.  A member
// claims the next round number; once the previous round is defined the new
// round starts where that one ends and takes up to kConsBatch messages that
// are already published (so a round never waits on room the ring cannot
// give); the member copies it and releases the ring room in round order.
// Each message's ring position and output address come from the record its
// producer wrote before publishing, so a member never needs another round's
// entries (which producers may already be reusing).
__device__ void run_lock_team(const PumpArgs &a, uint32_t uid, uint32_t tid) {
  __shared__ uint64_t s_pout[kMaxProducers], s_pbytes[kMaxProducers];
  __shared__ uint64_t s_pfirst[kMaxProducers], s_pn[kMaxProducers];
  __shared__ uint32_t s_psid[kMaxProducers];
  __shared__ uint64_t s_sz[kConsBatch], s_pos[kConsBatch], s_out[kConsBatch];
  __shared__ uint32_t s_p[kConsBatch], s_bad;
  __shared__ Seg s_seg[2 * kConsBatch];
  __shared__ uint64_t s_start, s_end, s_total_v, s_bend;
  __shared__ uint32_t s_stop, s_nseg;
  const DevChannel u = a.chans[uid];
  const DevRing r = a.rings[u.first_ring];
  const uint64_t tm_a = r.coord + offsetof(RingCoord, prod);
  const uint64_t hm_a = r.coord + offsetof(RingCoord, cons), hb_a = hm_a + 8;
  const uint64_t last = r.base_m + u.total_msgs;  // counter after this pump's messages
  uint64_t *rounds = (uint64_t *)u.rounds;
  for (uint32_t p = tid; p < u.K; p += kPumpBlock) {
    const uint32_t sid = a.stream_of_prod[u.prod_stream_base + p];
    const DevStream so = a.streams[sid];
    s_psid[p] = sid;
    s_pout[p] = so.out_base;
    s_pbytes[p] = so.out_bytes;
    s_pfirst[p] = so.first_msg;
    s_pn[p] = so.n_msgs;
  }
  Watch w{0, a.timeout_ticks, a.err, 0};
  w.progress();
  for (;;) {
    if (tid == 0) {
      uint32_t stop = 0;
      const uint64_t k = __hip_atomic_fetch_add((uint64_t *)u.claim, 1ull, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
      uint64_t start = r.base_m;
      if (k > 0) {
        uint64_t v;
        while ((v = ld_rlx((uint64_t)&rounds[k - 1])) == 0) {
          __builtin_amdgcn_s_sleep(1);
          if (w.expired()) {
            stop = 1;
            break;
          }
        }
        start = v - 1;
      }
      uint64_t end = start;
      if (!stop && start < last) {
        uint64_t tm;
        while ((tm = ld_rlx(tm_a)) <= start) {
          __builtin_amdgcn_s_sleep(2);
          if (w.expired()) {
            stop = 1;
            break;
          }
        }
        if (!stop) {
          end = start + kConsBatch;
          if (end > tm) end = tm;
          if (end > last) end = last;
        }
      }
      // round k is defined even when empty: later claimers see where it ends
      if (!stop) st_rlx((uint64_t)&rounds[k], end + 1);
      s_start = start;
      s_end = end;
      s_stop = stop || start >= last;
      s_bad = 0;
    }
    __syncthreads();
    if (s_stop) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // records and payload of the round
    const uint64_t start = s_start, n = s_end - s_start;
    if (tid < n) {
      const uint64_t seq = start + tid;
      const uint64_t e = *(const GLOBAL uint64_t *)(r.entries + 8 * (seq % r.E));
      const uint64_t *rec = (const uint64_t *)(r.side + 24 * (seq - r.base_m));
      const uint64_t sz = e & kEntrySizeMask, pos = rec[0], out = rec[1], mi = rec[2];
      const uint32_t p = (uint32_t)(e >> 48) % u.K;
      // checked against the producer's stream before any byte moves
      if (sz > r.P || out < s_pout[p] || out - s_pout[p] > s_pbytes[p] ||
          sz > s_pbytes[p] - (out - s_pout[p]) || mi < s_pfirst[p] || mi - s_pfirst[p] >= s_pn[p])
        atomicOr(&s_bad, 1u);
      s_sz[tid] = sz;
      s_pos[tid] = pos;
      s_out[tid] = out;
      s_p[tid] = p;
      if (a.trace) a.trace[u.trace_base + (seq - r.base_m)] = s_psid[p];
      if (a.ts_pop) a.ts_pop[mi] = wall_clock64();
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t nseg = 0;
      uint64_t v = 0;
      for (uint32_t i = 0; i < n; i++) {
        const uint64_t sz = s_sz[i], pos = s_pos[i] % r.P;
        const uint64_t first = r.P - pos < sz ? r.P - pos : sz;
        if (first) {
          s_seg[nseg] = make_seg(s_out[i], r.payload + pos, first);
          s_seg[nseg].v0 = v;
          v += s_seg[nseg++].nv;
        }
        if (sz > first) {
          s_seg[nseg] = make_seg(s_out[i] + first, r.payload, sz - first);
          s_seg[nseg].v0 = v;
          v += s_seg[nseg++].nv;
        }
      }
      s_nseg = nseg;
      s_total_v = v;
      s_bend = n ? s_pos[n - 1] + s_sz[n - 1] : 0;
      if (s_bad) {
        __hip_atomic_fetch_or(&a.err[0], kErrCorrupt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_stop = 1;
      }
    }
    __syncthreads();
    if (s_stop) break;
    seg_copy<kPumpBlock, 4>(s_seg, s_nseg, s_total_v, tid);
    __syncthreads();  // every read of the ring has completed
    if (tid == 0) {
      // release in round order
      while (ld_rlx(hm_a) != start) {
        __builtin_amdgcn_s_sleep(1);
        if (w.expired()) {
          s_stop = 1;
          break;
        }
      }
      if (!s_stop) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        st_rlx(hb_a, s_bend);
        st_rlx(hm_a, s_end);
      }
    }
    __syncthreads();
    if (s_stop) break;
    w.progress();
  }
  __threadfence();
}

__global__ __launch_bounds__(kPumpBlock) __attribute__((amdgpu_waves_per_eu(6, 8)))
void pump_kernel(PumpArgs a) {
  const DevRole role = a.roles[blockIdx.x];
  const uint32_t tid = threadIdx.x;
  __shared__ Seg s_pseg[4][2 * kProdBatch];
  if (role.kind == 0) {
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave
    if (wave < role.count) run_producer(a, a.roles[blockIdx.x].ids[wave], tid & 63, s_pseg[wave]);
    __threadfence();
  } else if (a.chans[role.ids[0]].mode == kModeMpscLock) {
    run_lock_team(a, role.ids[0], tid);
  } else {
    run_consumer(a, role.ids[0], tid);
  }
}

// Host-API push: copy the payload into the ring, write the entries, then
// publish the new message counter into host-coherent memory with a
// system-scope release.
__global__ __launch_bounds__(256) void push_kernel(PushArgs a) {
  const uint32_t tid = threadIdx.x;
  ring_put<256, 4>(a.ring, a.pos, a.src, a.bytes, tid);
  for (uint32_t i = tid; i < a.n_entries; i += 256)
    *(GLOBAL uint64_t *)(a.ring.entries + 8 * ((a.first_entry + i) % a.ring.E)) =
        a.entry_bytes | ((uint64_t)a.producer << 48);
  __threadfence_system();
  __syncthreads();
  if (tid == 0)
    __hip_atomic_store(a.publish, a.publish_value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_pump(const PumpArgs &a, uint32_t n_wgs, hipStream_t stream) {
  hipLaunchKernelGGL(pump_kernel, dim3(n_wgs), dim3(kPumpBlock), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_push(const PushArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(push_kernel, dim3(1), dim3(256), 0, stream, a);
  return hipGetLastError();
}

int pump_occupancy(int *wgs_per_cu) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, pump_kernel, kPumpBlock, 0);
}

}  // namespace hicr
